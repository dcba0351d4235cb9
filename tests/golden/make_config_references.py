"""Write the oracle's whole-run references of the two-species and the
relativistic beam workloads at their full sizes, by the CPU FP64 oracle only:

    python tests/golden/make_config_references.py c2      (about 3 minutes)
    python tests/golden/make_config_references.py c4      (about 40 minutes)

c2: 4096 cells of Poisson(256) electrons and ions (m_i/m_e = 100), 200 steps,
    N97 and TA77; per step T_e and T_i (weighted temperature about the
    species' mean velocity, averaged over the three components).
    Files tests/golden/c2_{n97,ta77}_relaxation_oracle.txt.
c4: 16384 cells of 448 background electrons, 128 beam electrons (weight
    1e-2, gamma = 3 along x) and 448 ions (m_i/m_e = 1836) in Maxwell-Juettner
    backgrounds (theta = 0.05), relativistic N97, 500 steps; per step the
    beam's mean proper velocity along x and mean kinetic energy, and the mean
    kinetic energies of the background electrons and of the ions (weighted,
    per unit weight, c = 1).  File tests/golden/c4_beam_oracle.txt.

Each file holds the run with the workload's own Philox seed and, as the scale
of what the collision noise alone moves, the same run with the seed + 1 and
+ 2 (the initial population unchanged).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2407_19151_amd import workloads as W  # noqa: E402

N_ALT = 2


def c2_observables(wl):
    out = []
    for sp in range(wl.n_species):
        k = wl.species == sp
        w = wl.w[k]
        v = np.stack([wl.vx[k], wl.vy[k], wl.vz[k]])
        mean = (v * w).sum(1, keepdims=True) / w.sum()
        out.append(wl.mass[sp] * (w * ((v - mean) ** 2).sum(0)).sum() / (3.0 * w.sum()))
    return out


def c4_masks(wl):
    # beam electrons carry 1e-2 of a background electron's weight
    e = wl.species == 0
    wmax = wl.w[e].max()
    beam = e & (wl.w < 0.5 * wmax)
    return beam, e & ~beam, wl.species == 1


def c4_observables(wl, masks):
    u2 = wl.vx ** 2 + wl.vy ** 2 + wl.vz ** 2
    kin = wl.mass[wl.species] * u2 / (np.sqrt(1.0 + u2) + 1.0)  # m (gamma - 1), c = 1
    beam, bg, ion = masks
    out = [float((wl.w[beam] * wl.vx[beam]).sum() / wl.w[beam].sum())]
    for m in (beam, bg, ion):
        out.append(float((wl.w[m] * kin[m]).sum() / wl.w[m].sum()))
    return out


def run(make, observe, steps, seed_offset):
    wl = make()
    wl.seed = wl.seed + seed_offset
    rows = [observe(wl)]
    t0 = time.time()
    for k in range(steps):
        oracle.run_workload(wl, steps=1, first_step=k)
        rows.append(observe(wl))
        if (k + 1) % 50 == 0:
            print("  seed +%d: %d/%d steps, %.0f s" % (seed_offset, k + 1, steps, time.time() - t0),
                  flush=True)
    return np.array(rows), wl


def write(path, header, runs):
    steps = runs[0].shape[0]
    with open(path, "w") as f:
        for line in header:
            f.write("# " + line + "\n")
        f.write("# written by tests/golden/make_config_references.py (oracle only)\n")
        for k in range(steps):
            f.write("%d " % k + " ".join("%.17e" % x for r in runs for x in r[k]) + "\n")


def main():
    oracle.set_threads(os.cpu_count() or 1)
    what = sys.argv[1:] or ["c2", "c4"]
    if "c2" in what:
        for name, method in (("n97", W.N97), ("ta77", W.TA77)):
            runs = []
            for off in range(1 + N_ALT):
                r, wl = run(lambda: W.config2(method=method), c2_observables, 200, off)
                runs.append(r)
            write(os.path.join(HERE, "c2_%s_relaxation_oracle.txt" % name),
                  ["oracle (CPU FP64): config2(method=%s), %d cells, %d particles, 200 steps"
                   % (name.upper(), wl.n_cells, wl.n),
                   "columns: step, then (T_e, T_i) for the Philox seed + 0, + 1, + 2"], runs)
    if "c4" in what:
        runs = []
        for off in range(1 + N_ALT):
            base = W.config4()
            masks = c4_masks(base)
            r, wl = run(W.config4, lambda x: c4_observables(x, masks), 500, off)
            runs.append(r)
        write(os.path.join(HERE, "c4_beam_oracle.txt"),
              ["oracle (CPU FP64): config4(), %d cells, %d particles, relativistic N97, 500 steps"
               % (wl.n_cells, wl.n),
               "columns: step, then (beam <u_x>, beam <KE>, background-electron <KE>, ion <KE>)"
               " per unit weight for the Philox seed + 0, + 1, + 2"], runs)


if __name__ == "__main__":
    main()
