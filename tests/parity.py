"""Comparison helpers shared by the GPU parity tests (no device work here).

Eigenvectors are compared as subspaces: the levels of a window are grouped
into clusters whose neighbouring gaps are below GAP_MIN ||H|| (a cluster of one
is an isolated level); for each GPU cluster the singular values of
Psi_oracle^T Psi_gpu, with Psi_oracle the oracle's eigenvectors of the same
energies (whole clusters, from a window wide enough to hold a cluster cut by
the window edge), must all be at least 1 - SUB_TOL.  For an isolated level this
is |<psi_o|psi_g>| >= 1 - SUB_TOL.  Where the levels of a cluster are exactly
degenerate any basis of the cluster is an answer, and this is what is unique.
"""
import numpy as np

GAP_MIN = 1e-6      # levels closer than GAP_MIN ||H|| form a cluster
SUB_TOL = 1e-8


def clusters(E, hn, gap_min=GAP_MIN):
    """Index groups of consecutive ascending levels with gaps below gap_min hn."""
    E = np.asarray(E)
    if E.size == 0:
        return []
    out, cur = [], [0]
    for i in range(1, E.size):
        if E[i] - E[i - 1] < gap_min * hn:
            cur.append(i)
        else:
            out.append(cur)
            cur = [i]
    out.append(cur)
    return out


def subspace_cosines(Eg, Zg, Eo, Zo, hn, eig_tol=1e-10):
    """For every cluster of the GPU window (Eg ascending, Zg dim x nev), the
    smallest singular value of Zo_c^T Zg_c, where Zo_c are the oracle vectors of
    every oracle cluster (of the ascending oracle window Eo, Zo) meeting the
    cluster's energy range.  Returns a list of (indices, min singular value)."""
    oc = clusters(Eo, hn)
    res = []
    for grp in clusters(Eg, hn):
        lo, hi = Eg[grp[0]] - eig_tol * hn, Eg[grp[-1]] + eig_tol * hn
        cols = [i for c in oc if Eo[c[-1]] >= lo and Eo[c[0]] <= hi for i in c]
        if len(cols) < len(grp):
            res.append((grp, 0.0))
            continue
        s = np.linalg.svd(Zo[:, cols].T @ Zg[:, grp], compute_uv=False)
        res.append((grp, float(s.min())))
    return res


def assert_subspaces(Eg, Zg, Eo, Zo, hn, tol=SUB_TOL):
    bad = [(g, s) for g, s in subspace_cosines(Eg, Zg, Eo, Zo, hn) if s < 1.0 - tol]
    assert not bad, f"clusters not matched as subspaces: {bad[:4]}"


def kl_tolerance(Z, E, resid_oracle, hn):
    """Tolerance of KL(p_k || p_k+1) for GPU vectors whose residuals the oracle
    computed (resid_oracle[k] = ||H psi_k - E_k psi_k||, H applied by the
    oracle).  KL is ill-conditioned where components of the neighbour are tiny;
    its first-order error for a componentwise vector error delta (Davis-Kahan:
    residual / gap to the other levels) is est = sum_i p_i min(1, 2 delta /
    |phi_i|) + sum_i |ln(p_i / q_i)| min(p_i, 2 delta |psi_i|); the tolerance is
    1e-7 + 10 est."""
    nev = Z.shape[1]
    ktol = np.full(nev - 1, 1e-7)
    for k in range(nev - 1):
        gaps_k = [abs(E[k + 1] - E[k])]
        if k > 0:
            gaps_k.append(abs(E[k] - E[k - 1]))
        if k + 2 < nev:
            gaps_k.append(abs(E[k + 2] - E[k + 1]))
        delta = max(resid_oracle[k], resid_oracle[k + 1]) / max(min(gaps_k), 1e-300) + 1e-14
        psi, phi = np.abs(Z[:, k]), np.abs(Z[:, k + 1])
        p_, q_ = psi ** 2, phi ** 2
        nz = (phi > 0) & (psi > 0)
        est = np.sum(p_[phi > 0] * np.minimum(1.0, 2 * delta / phi[phi > 0]))
        est += np.sum(np.abs(np.log(p_[nz] / q_[nz])) * np.minimum(p_[nz], 2 * delta * psi[nz]))
        ktol[k] += 10.0 * est
    return ktol
