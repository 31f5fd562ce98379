"""Write the stored oracle values used by the full-size parity checks.

Calls only the Ewald oracle (oracle/) and the seeded input generators; no
value here comes from the GPU library.  Run from the repository root:

    python tests/golden/make_golden.py shell3d     # N = 1e7 thin shell, 64 targets
    python tests/golden/make_golden.py clustered3d # N = 1e6 clustered triclinic, 64 targets
    python tests/golden/make_golden.py clustered3d_grad  # same, potential and gradient
    python tests/golden/make_golden.py shell3d_bloch  # N = 1e7 shell, Bloch conditions
    python tests/golden/make_golden.py paper [name ...]  # the paper's nine cells, N = 1e7

Each output file has one line per sampled target: the source index and the
tin-foil potential there (targets = sources, self pair removed); the _grad
file adds the d components of grad Phi; the _bloch file holds the real and
imaginary parts of the quasi-periodic potential for the Bloch vector BLOCH.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ewald  # noqa: E402
from paper_2606_28608_amd import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
NSAMPLE = 64
SAMPLE_SEED = 123
BLOCH = np.array([0.7, -1.1, 0.4])   # Bloch vector of the stored quasi-periodic values


def sample(n):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, NSAMPLE, replace=False))


def write(name, L, src, q, header):
    idx = sample(len(q))
    pot = ewald.ewald_sampled(L, src, q, idx)
    path = os.path.join(HERE, name)
    np.savetxt(path, np.c_[idx, pot], fmt=["%d", "%.17e"], header=header)
    print("wrote", path)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "shell3d"
    if which == "shell3d":
        L, src, q = workloads.shell3d(10_000_000, seed=3)
        write("shell3d_n1e7_seed3.txt", L, src, q,
              "workloads.shell3d(10_000_000, seed=3); oracle Ewald at 64 sampled sources "
              "(numpy default_rng(123).choice); columns: index potential")
    elif which == "clustered3d_grad":
        L, src, q = workloads.clustered3d(1_000_000, seed=2)
        idx = sample(len(q))
        pot, grad = ewald.ewald_sampled(L, src, q, idx, grad=True)
        path = os.path.join(HERE, "clustered3d_n1e6_seed2_grad.txt")
        np.savetxt(path, np.c_[idx, pot, grad], fmt=["%d"] + ["%.17e"] * 4,
                   header="workloads.clustered3d(1_000_000, seed=2); oracle Ewald potential and "
                          "gradient at 64 sampled sources (numpy default_rng(123).choice); "
                          "columns: index potential gx gy gz")
        print("wrote", path)
    elif which == "shell3d_bloch":
        L, src, q = workloads.shell3d(10_000_000, seed=3)
        idx = sample(len(q))
        pot = ewald.ewald_bloch_sampled(L, src, q, BLOCH, idx)
        path = os.path.join(HERE, "shell3d_n1e7_seed3_bloch.txt")
        np.savetxt(path, np.c_[idx, pot.real, pot.imag], fmt=["%d", "%.17e", "%.17e"],
                   header="workloads.shell3d(10_000_000, seed=3); oracle Bloch Ewald with "
                          "beta = (0.7, -1.1, 0.4) at 64 sampled sources (numpy "
                          "default_rng(123).choice); columns: index re im")
        print("wrote", path)
    elif which == "paper":
        names = sys.argv[2:] or list(workloads.PAPER_SYSTEMS)
        for name in names:
            L, src, q = workloads.paper_system(name, 10_000_000)
            write("paper_%s_n1e7_seed8.txt" % name, L, src, q,
                  "workloads.paper_system(%r, 10_000_000) (seed 8); oracle Ewald at 64 sampled "
                  "sources (numpy default_rng(123).choice); columns: index potential" % name)
    elif which == "clustered3d":
        L, src, q = workloads.clustered3d(1_000_000, seed=2)
        write("clustered3d_n1e6_seed2.txt", L, src, q,
              "workloads.clustered3d(1_000_000, seed=2); oracle Ewald at 64 sampled sources "
              "(numpy default_rng(123).choice); columns: index potential")
