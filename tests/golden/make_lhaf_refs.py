"""Writes tests/golden/lhaf_refs_ld.txt: long-double oracle values of full
power-trace subset sums (Sec. IV) for the workloads whose full sums are too
slow to recompute inside a GPU test.

Only the oracle and the seeded input recipes are used.  Each line is
    name  N  re  im  sum_S|t_S|
with the long-double values printed to 21 significant digits.  Run from the
repository root:
    python tests/golden/make_lhaf_refs.py [name ...]
(no names: every reference; existing lines of other names are kept).

Names:
    c3_<N>      the M = 100, r = 1.2 state with N distinct modes (N = 40, 44, 50)
    c4_<i>      item i of the 4096-item chain-like batch workload
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2010_15595_amd import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lhaf_refs_ld.txt")


def c4_picks(dims):
    """One item of every even N in 22..36 (the lowest index) and the eight
    largest items (stable order), as the batch parity test selects them."""
    dims = np.asarray(dims)
    pick = []
    for N in range(22, 37, 2):
        idx = np.nonzero(dims == N)[0]
        if len(idx):
            pick.append(int(idx[0]))
    pick += [int(i) for i in np.argsort(dims, kind="stable")[-8:]]
    return sorted(set(pick))


def c4_matrices():
    st = workloads.config4(count=4096)
    return [oracle.expand(st["B"], st["gamma"], pat) for pat in st["patterns"]]


def all_names():
    dims = [a.shape[0] for a in c4_matrices()]
    return ["c3_40", "c3_44", "c3_50"] + [f"c4_{i}" for i in c4_picks(dims)]


def matrix(name, c4=None):
    kind, arg = name.split("_")
    if kind == "c3":
        st = workloads.config3(int(arg))
        return oracle.expand(st["B"], st["gamma"], st["pattern"])
    if kind == "c4":
        return (c4 if c4 is not None else c4_matrices())[int(arg)]
    raise ValueError(name)


def load(path=OUT):
    """{name: (N, re, im, abs_sum)} with np.longdouble values."""
    refs = {}
    if not os.path.exists(path):
        return refs
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, N, re, im, ab = line.split()
            refs[name] = (int(N), np.longdouble(re), np.longdouble(im), np.longdouble(ab))
    return refs


def fmt(x):
    return np.format_float_scientific(np.longdouble(x), precision=20, unique=False)


def main(names):
    refs = load()
    c4 = c4_matrices()
    for name in names:
        A = matrix(name, c4)
        t = time.time()
        (re, im), ab = oracle.lhaf_pt(A, prec="ld", with_abs=True)
        refs[name] = (A.shape[0], re, im, ab)
        print(f"{name}: N={A.shape[0]} {fmt(re)} {fmt(im)} sum|t|={fmt(ab)} ({time.time() - t:.1f} s, "
              f"{oracle.max_threads()} threads)", flush=True)
        with open(OUT + ".tmp", "w") as f:
            f.write("# long-double oracle full sums: name N re im sum_S|t_S| (tests/golden/make_lhaf_refs.py)\n")
            for k in sorted(refs):
                N, r, i, a = refs[k]
                f.write(f"{k} {N} {fmt(r)} {fmt(i)} {fmt(a)}\n")
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:] or all_names())
