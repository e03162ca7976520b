"""Writes cylinder_s025_wall_sums.txt: the oracle's surface sums of the
reduced Mach 10 cylinder (scale 0.25: 150 x 75 cells of the full grid's
1-mm size, ~2.25M particles, FP32 state, seed 99, capacity 1.6x the initial
fill, so that no injection is dropped), sampled over steps 1000..2999 after
1000 steps of flow development, 36 body elements (Sec. V.C sampling).  One row per surface element (walls, then the body), the nine
fixed-point sums of the surface sampling.  Calls only the oracle and the
seeded workload generators.

    PYTHONPATH=. python tests/golden/make_cylinder_wall_sums.py   (about 30 min on 8 threads)
"""
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))
import oracle  # noqa: E402
import usp_workloads as W  # noqa: E402

SCALE, TRANSIENT, SAMPLED, NBODY = 0.25, 1000, 2000, 36
OUT = os.path.join(os.path.dirname(__file__), "cylinder_s025_wall_sums.txt")


def main():
    prob = W.cylinder(scale=SCALE, f32=True)
    sim = oracle.Sim(prob, W.particles_for(prob))
    sim.step_native(0, TRANSIENT)
    sim.enable_sampling(NBODY)
    sim.step_native(TRANSIENT, SAMPLED)
    dropped = sim.cnt()["CAPACITY"]
    if dropped:
        raise SystemExit(f"{dropped} injections dropped for lack of capacity")
    with open(OUT, "w") as f:
        f.write("# Oracle surface sums of the scale-0.25 Mach 10 cylinder (FP32 state, seed 99,\n")
        f.write(f"# capacity {sim.cap} for {sim.n} particles at the end, no injection dropped),\n")
        f.write(f"# steps {TRANSIENT}..{TRANSIENT + SAMPLED - 1}, {NBODY} body elements; written by\n")
        f.write("# tests/golden/make_cylinder_wall_sums.py (oracle only).  Columns: "
                + " ".join(oracle.SURF_NAMES) + "\n")
        for row in sim.surf:
            f.write(" ".join(str(int(v)) for v in row) + "\n")


if __name__ == "__main__":
    main()
