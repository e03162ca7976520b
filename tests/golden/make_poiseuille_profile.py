"""Writes poiseuille_kn005_200x1000.txt and poiseuille_kn001_200x1000.txt:
the oracle's time-averaged velocity profile of the force-driven channel
(Sec. V.B) at full size, 200 cells x 1000 particles with an FP32 state,
seed 7, at Kn = 0.05 and Kn = 0.01: the transient steps (2000 and 4500; the
viscous decay is five times slower at Kn = 0.01), then the field sums of
the next 4000 (each taken on the binned state after a step).  Calls only
the oracle and the seeded workload generators.

    PYTHONPATH=. python tests/golden/make_poiseuille_profile.py [kn]   (4-5 min each)
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))
import oracle  # noqa: E402
import usp_workloads as W  # noqa: E402

CELLS, PPC, SAMPLED = 200, 1000, 4000
RUNS = {0.05: (2000, "poiseuille_kn005_200x1000.txt"), 0.01: (4500, "poiseuille_kn001_200x1000.txt")}


def main(kn):
    TRANSIENT, name = RUNS[kn]
    OUT = os.path.join(os.path.dirname(__file__), name)
    prob = W.poiseuille(kn=kn, cells=CELLS, ppc=PPC, f32=True)
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
        f.write(f"# Oracle time average of the Kn = {kn} channel, 200 cells x 1000 particles,\n")
        f.write(f"# FP32 state, seed 7, steps {TRANSIENT}..{TRANSIENT + SAMPLED - 1} sampled; written by\n")
        f.write("# tests/golden/make_poiseuille_profile.py (oracle only).\n")
        f.write(f"T_tr {T:.6f}\n")
        f.write("# cell  U_x [m/s]\n")
        for k, u in enumerate(U):
            f.write(f"{k} {u:.9e}\n")


if __name__ == "__main__":
    for kn in ([float(sys.argv[1])] if len(sys.argv) > 1 else sorted(RUNS)):
        main(kn)
