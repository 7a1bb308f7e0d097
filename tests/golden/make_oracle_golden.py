"""Writes the stored oracle results used by the GPU parity tests at sizes where
the dense oracle takes minutes (L = 14, 16).  Calls only ``oracle/``.

    python tests/golden/make_oracle_golden.py [--L 14 16] [--procs 5]

Each output file ``oracle_L{L}_h{h}_s{seed}.json`` holds, for one disorder
realization (fields from SplitMix64(seed)), the extremal energies and, for each
target eps in {0.1, 0.3, 0.5, 0.7, 0.9}, the 50 eigenvalues nearest
sigma = E_min + eps (E_max - E_min) with r, S_1, S_2, S_E, F, f and KL.  At
L = 14 each target also stores the oracle eigenvectors of the clusters of levels
closer than 1e-6 ||H|| to a neighbour that are cut by the window edge, and of
the one nearest sigma inside it (key "clusters": energies and vectors of the
whole cluster, taken from a window of nev + 8 levels so a cluster cut by the
window edge is complete), so that the GPU's vectors there can be compared as
subspaces.  The clean chain (h = 0) is
one of the L = 14 realizations: its translation and reflection symmetries
make exactly degenerate levels.
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

EPS = [0.1, 0.3, 0.5, 0.7, 0.9]
NEV = 50
CLUSTER_REL = 1e-6          # levels closer than this times ||H|| form a cluster
CLUSTER_VECTORS_L = (14,)   # sizes whose goldens carry the cluster vectors


def clusters(evals, hnorm):
    """Groups of consecutive window indices whose neighbouring gaps are below
    CLUSTER_REL ||H|| (groups of one are left out)."""
    out, cur = [], [0]
    for i in range(1, len(evals)):
        if evals[i] - evals[i - 1] < CLUSTER_REL * hnorm:
            cur.append(i)
        else:
            if len(cur) > 1:
                out.append(cur)
            cur = [i]
    if len(cur) > 1:
        out.append(cur)
    return out

CASES = {
    14: [(h, s) for h in (1.0, 3.0, 5.0) for s in (0, 1)] + [(0.0, 0)],
    16: [(h, 0) for h in (1.0, 2.0, 3.0, 4.0, 5.0)] + [(3.0, 1)],
}


def _one(args):
    L, h, seed = args
    path = os.path.join(HERE, f"oracle_L{L}_h{h:.1f}_s{seed}.json")
    if os.path.exists(path):
        return path, 0.0
    t0 = time.time()
    want_vec = L in CLUSTER_VECTORS_L
    outs = oracle.solve_targets(L, h, seed, EPS, NEV)
    wide = (oracle.solve_targets(L, h, seed, EPS, NEV + 8, observables=False, vectors=True)
            if want_vec else None)
    rec = dict(L=L, h=h, seed=seed, J=1.0, nev=NEV, fields=outs[0]["fields"].tolist(),
               emin=outs[0]["emin"], emax=outs[0]["emax"], targets=[])
    for o in outs:
        rec["targets"].append({k: (v.tolist() if hasattr(v, "tolist") else v)
                               for k, v in o.items()
                               if k in ("eps", "sigma", "evals", "r", "r_mean", "s1", "s2",
                                        "se", "fluct", "dynfrac", "kl")})
        if want_vec:
            w = wide[len(rec["targets"]) - 1]
            lo, hi = o["evals"][0], o["evals"][-1]
            pad = CLUSTER_REL * o["hnorm"]
            meet = [c for c in clusters(w["evals"], o["hnorm"])
                    if w["evals"][c[-1]] >= lo - pad and w["evals"][c[0]] <= hi + pad]
            # to keep the fixture small: every cluster cut by the window edge
            # and the interior cluster nearest sigma
            edge = [c for c in meet if w["evals"][c[0]] < lo + pad or w["evals"][c[-1]] > hi - pad]
            inner = sorted((c for c in meet if c not in edge),
                           key=lambda c: abs(w["evals"][c[0]] - o["sigma"]))[:1]
            rec["targets"][-1]["clusters"] = [
                {"evals": [float(w["evals"][i]) for i in c],
                 "vecs": [w["evecs"][:, i].tolist() for i in c]}
                for c in edge + inner]
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(rec, fh)
    os.replace(tmp, path)
    return path, time.time() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, nargs="*", default=[14, 16])
    ap.add_argument("--procs", type=int, default=5)
    a = ap.parse_args()
    oracle.build(force=False)
    jobs = [(L, h, s) for L in a.L for (h, s) in CASES[L]]
    with Pool(a.procs) as pool:
        for path, dt in pool.imap_unordered(_one, jobs):
            print(f"{os.path.basename(path)} {dt:.1f}s", flush=True)


if __name__ == "__main__":
    main()
