"""Writes poiseuille_kn005_200x1000.txt: the oracle's time-averaged
velocity profile of the Kn = 0.05 force-driven channel (Sec. V.B) at full
size, 200 cells x 1000 particles with an FP32 state, seed 7: 2000 transient
steps, then the field sums of the next 4000 (each taken on the binned state
after a step).  Calls only the oracle and the seeded workload generators.

    PYTHONPATH=. python tests/golden/make_poiseuille_profile.py   (about 4 min)
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))
import oracle  # noqa: E402
import usp_workloads as W  # noqa: E402

CELLS, PPC, TRANSIENT, SAMPLED = 200, 1000, 2000, 4000
OUT = os.path.join(os.path.dirname(__file__), "poiseuille_kn005_200x1000.txt")


def main():
    prob = W.poiseuille(kn=0.05, cells=CELLS, ppc=PPC, f32=True)
    sim = oracle.Sim(prob, W.particles_for(prob))
    sim.enable_sampling()
    sim.step_native(0, TRANSIENT)
    for s in range(SAMPLED):
        sim.step_native(TRANSIENT + s, 1)
        sim.bin()
        sim.sample_fields()
    F = sim.fields
    i = oracle.SAMP_NAMES.index
    N, cx = F[i("N")], F[i("CX")]
    U = cx / N
    # translational temperature: 3 R T = <|c - U|^2>
    c2 = F[i("CXX")] + F[i("CYY")] + F[i("CZZ")]
    cu = (cx ** 2 + F[i("CY")] ** 2 + F[i("CZ")] ** 2) / N
    T = (c2 - cu).sum() / N.sum() / (3 * prob.gas.R)
    with open(OUT, "w") as f:
        f.write("# Oracle time average of the Kn = 0.05 channel, 200 cells x 1000 particles,\n")
        f.write("# FP32 state, seed 7, steps 2000..5999 sampled; written by\n")
        f.write("# tests/golden/make_poiseuille_profile.py (oracle only).\n")
        f.write(f"T_tr {T:.6f}\n")
        f.write("# cell  U_x [m/s]\n")
        for k, u in enumerate(U):
            f.write(f"{k} {u:.9e}\n")


if __name__ == "__main__":
    main()
