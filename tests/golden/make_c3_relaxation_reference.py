"""Write the oracle's relaxation reference for the FP32-kinematics rate check:
electron and ion temperatures after each of 200 steps of 4096 cells of the
uneven-cell workload's recipe (lognormal counts clipped to [16, 4096],
electrons and ions, m_i/m_e = 100, N97, moment correction), by the CPU FP64
oracle only.

    python tests/golden/make_c3_relaxation_reference.py

Output: tests/golden/c3_4096_relaxation_oracle.txt, one line per step:
step, T_e, T_i (weighted temperature about the species' mean velocity,
averaged over the three components).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2407_19151_amd import workloads as W  # noqa: E402

N_CELLS, STEPS = 4096, 200
OUT = os.path.join(HERE, "c3_4096_relaxation_oracle.txt")


def temperatures(wl):
    out = []
    for sp in range(wl.n_species):
        k = wl.species == sp
        w = wl.w[k]
        v = np.stack([wl.vx[k], wl.vy[k], wl.vz[k]])
        mean = (v * w).sum(1, keepdims=True) / w.sum()
        out.append(wl.mass[sp] * (w * ((v - mean) ** 2).sum(0)).sum() / (3.0 * w.sum()))
    return out


def main():
    oracle.set_threads(os.cpu_count() or 1)
    wl = W.config3(n_cells=N_CELLS)
    rows = [(0, *temperatures(wl))]
    for k in range(STEPS):
        oracle.run_workload(wl, steps=1, first_step=k)
        rows.append((k + 1, *temperatures(wl)))
    with open(OUT, "w") as f:
        f.write("# oracle (CPU FP64): %d cells of the uneven-cell recipe (config3(n_cells=%d), "
                "%d particles), %d steps\n" % (N_CELLS, N_CELLS, wl.n, STEPS))
        f.write("# written by tests/golden/make_c3_relaxation_reference.py\n")
        f.write("# step T_e T_i\n")
        for r in rows:
            f.write("%d %.17e %.17e\n" % r)


if __name__ == "__main__":
    main()
