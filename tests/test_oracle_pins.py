"""Pins of the CPU oracle against facts that do not come from the oracle itself:
the paper's printed numbers, closed forms of the model, an independent
brute-force construction of the full 2^L Hamiltonian, textbook spectra, LAPACK
(numpy) as an independent eigensolver, and symmetry invariants.  Each pin is
chosen so that a plausible slip (dropped term, wrong sign or index, transposed
operand, a missing ln 2) fails it."""
import math
import os

import numpy as np
import pytest

import oracle
from conftest import GOLDEN

# ----------------------------------------------------------------- generator

def test_splitmix64_published_sequence():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) as fh:
        vals = [int(x) for x in fh.read().split("\n") if x and x[0].isdigit()]
    assert oracle.splitmix64(1234567, 5) == vals
    assert oracle.splitmix64(0, 1)[0] == 0xE220A8397B1DCDAF


def test_fields_uniform_in_range_and_mean():
    f = np.concatenate([oracle.fields(1000, 2.5, s) for s in range(20)])
    assert f.min() >= -2.5 and f.max() < 2.5
    # U[-h, h]: mean 0, variance h^2/3
    assert abs(f.mean()) < 0.05
    assert abs(f.var() - 2.5 ** 2 / 3) < 0.05


# ------------------------------------------------------------------- basis

@pytest.mark.parametrize("L", [2, 4, 6, 8, 10, 12, 14, 16])
def test_sector_dimension_and_order(L):
    b = oracle.basis(L)
    assert b.size == math.comb(L, L // 2)
    assert np.all(np.diff(b.astype(np.int64)) > 0)
    assert all(bin(int(s)).count("1") == L // 2 for s in b[:: max(1, b.size // 97)])
    for k in range(0, b.size, max(1, b.size // 50)):
        assert oracle.rank(b, int(b[k])) == k


def test_sector_dimension_L22_printed_in_paper():
    # section "Numerical method" / introduction: dim H_{L=22} = 705 432 (S^z = 0)
    assert oracle.basis(22).size == 705432


# ----------------------------------------------- brute-force 2^L Hamiltonian

def _full_H(L, J, f):
    """Full 2^L matrix from Kronecker products of spin-1/2 matrices; site i is
    bit i (value 1 = up).  Complex S^y on purpose: nothing shared with the
    oracle's bit-flip construction."""
    sp = np.array([[0, 0], [1, 0]], dtype=complex)    # |0> -> |1>, raises S^z
    sm = sp.T.copy()
    sx = (sp + sm) / 2
    sy = (sp - sm) / 2j
    sz = np.diag([-0.5, 0.5]).astype(complex)

    def op(o, i):
        return np.kron(np.kron(np.eye(2 ** (L - 1 - i)), o), np.eye(2 ** i))

    n = 2 ** L
    H = np.zeros((n, n), dtype=complex)
    for i in range(L):
        j = (i + 1) % L
        for o in (sx, sy, sz):
            H += J * op(o, i) @ op(o, j)
        H += f[i] * op(sz, i)
    return H


@pytest.mark.parametrize("L", [2, 4, 6, 8])
def test_sector_block_equals_bruteforce(L):
    f = oracle.fields(L, 2.0, 11)
    Hf = _full_H(L, 1.0, f)
    assert np.abs(Hf.imag).max() < 1e-14
    Hf = Hf.real
    sz = sum(np.kron(np.kron(np.eye(2 ** (L - 1 - i)), np.diag([-0.5, 0.5])), np.eye(2 ** i))
             for i in range(L))
    assert np.abs(Hf @ sz - sz @ Hf).max() < 1e-13          # S^z_tot conserved
    b = oracle.basis(L)
    Hs = oracle.dense_H(L, 1.0, f, b)
    assert np.abs(Hf[np.ix_(b, b)] - Hs).max() < 1e-14
    # the sector spectrum is contained in the full spectrum
    wf = np.linalg.eigvalsh(Hf)
    for lam in oracle.eigvalsh(Hs):
        assert np.min(np.abs(wf - lam)) < 1e-12


def test_full_bruteforce_L10_spectrum():
    L = 10
    f = oracle.fields(L, 1.5, 3)
    Hf = _full_H(L, 1.0, f).real
    b = oracle.basis(L)
    w_block = np.linalg.eigvalsh(Hf[np.ix_(b, b)])
    w_or = oracle.eigvalsh(oracle.dense_H(L, 1.0, f, b))
    assert np.abs(w_block - w_or).max() < 1e-12


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("L", [4, 6, 8, 10, 12])
@pytest.mark.parametrize("J", [1.0, 0.7])
def test_trace_closed_forms(L, J):
    f = oracle.fields(L, 3.0, L)
    H = oracle.dense_H(L, J, f)
    dim = math.comb(L, L // 2)
    # the field term is traceless in the sector; each bond contributes -J/4
    # times (fraction of antiparallel minus parallel) ...
    tr = -J * dim * L / (4 * (L - 1))
    tr2 = dim * (3 * J * J * L * L / 16 + (L * np.sum(f ** 2) - np.sum(f) ** 2) / 4) / (L - 1)
    assert abs(np.trace(H) - tr) < 1e-10 * dim
    assert abs(np.sum(H * H) - tr2) < 1e-9 * abs(tr2)
    w = oracle.eigvalsh(H)
    assert abs(w.sum() - tr) < 1e-9 * dim
    assert abs((w ** 2).sum() - tr2) < 1e-9 * abs(tr2)


@pytest.mark.parametrize("seed", range(5))
def test_L2_spectrum(seed):
    f = oracle.fields(2, 3.0, seed)
    for J in (1.0, 0.3):
        w = oracle.eigvalsh(oracle.dense_H(2, J, f))
        rt = math.sqrt(J * J + ((f[0] - f[1]) / 2) ** 2)
        assert np.allclose(w, [-J / 2 - rt, -J / 2 + rt], atol=1e-14)


def test_L4_uniform_field_spectrum():
    for hz in (0.0, 0.9):
        w = oracle.eigvalsh(oracle.dense_H(4, 1.0, np.full(4, hz)))
        assert np.allclose(w, [-2, -1, 0, 0, 0, 1], atol=1e-13)


def test_J0_diagonal_limit():
    L = 10
    f = oracle.fields(L, 2.0, 7)
    b = oracle.basis(L)
    H = oracle.dense_H(L, 0.0, f, b)
    assert np.abs(H - np.diag(np.diag(H))).max() == 0.0
    exp = np.array([0.5 * sum(f[i] * (1 if (int(s) >> i) & 1 else -1) for i in range(L)) for s in b])
    assert np.allclose(np.diag(H), exp, atol=1e-14)
    out = oracle.solve(L, 2.0, 7, 0.5, 8, J=0.0)
    # basis-state eigenvectors: S_1 = S_E = 0
    assert np.allclose(out["s1"], 0, atol=1e-12)
    assert np.allclose(out["se"], 0, atol=1e-12)


# -------------------------------------------------------- eigensolver pins

def test_tridiagonal_ql_laplacian_closed_form():
    n = 200
    w = oracle.tridiag_eigvals(np.full(n, 2.0), np.full(n - 1, -1.0))
    k = np.arange(1, n + 1)
    exact = np.sort(2 - 2 * np.cos(k * np.pi / (n + 1)))
    assert np.abs(w - exact).max() < 1e-13


@pytest.mark.parametrize("n", [1, 2, 3, 17, 120])
def test_eigvalsh_vs_lapack_random(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    A = A + A.T
    assert np.abs(oracle.eigvalsh(A) - np.linalg.eigvalsh(A)).max() < 1e-12 * max(1, np.abs(A).max() * n)


def test_eigh_full_and_invit_agree():
    L = 8
    f = oracle.fields(L, 2.5, 1)
    H = oracle.dense_H(L, 1.0, f)
    w, Z = oracle.eigh_full(H)
    assert np.abs(H @ Z - Z * w).max() < 1e-12
    assert np.abs(Z.T @ Z - np.eye(H.shape[0])).max() < 1e-12
    out = oracle.nearest_eigenpairs(H, 0.5, 10)
    idx = np.argsort(np.abs(w - out["sigma"]))[:10]
    idx = idx[np.argsort(w[idx])]
    assert np.abs(w[idx] - out["evals"]).max() < 1e-13
    # inverse-iteration vectors equal the accumulated ones up to sign
    ov = np.abs(np.sum(Z[:, idx] * out["evecs"], axis=0))
    assert np.all(ov > 1 - 1e-10)


@pytest.mark.parametrize("L,h,eps", [(10, 1.0, 0.5), (12, 3.0, 0.5), (12, 5.0, 0.1), (12, 0.5, 0.9)])
def test_nearest_eigenpairs_vs_lapack(L, h, eps):
    out = oracle.solve(L, h, 0, eps, 20, observables=False)
    H = oracle.dense_H(L, 1.0, out["fields"])
    w = np.linalg.eigvalsh(H)
    assert abs(out["emin"] - w[0]) < 1e-12 and abs(out["emax"] - w[-1]) < 1e-12
    sig = w[0] + eps * (w[-1] - w[0])
    sel = np.sort(w[np.argsort(np.abs(w - sig), kind="stable")[:20]])
    assert np.abs(sel - out["evals"]).max() < 1e-12
    Z = out["evecs"]
    assert np.abs(H @ Z - Z * out["evals"]).max() < 1e-11
    assert np.abs(Z.T @ Z - np.eye(20)).max() < 1e-11


def test_selection_tie_break_lower_first():
    # eigenvalues 0..5 of a diagonal matrix, sigma = 2.5: 2 and 3 tie, then 1 and 4
    H = np.diag(np.arange(6.0))
    out = oracle.nearest_eigenpairs(H, 0.5, 3)
    assert out["sigma"] == 2.5
    assert list(out["evals"]) == [1.0, 2.0, 3.0]


# ---------------------------------------------------------------- symmetry

def test_spin_flip_reflection_translation():
    L = 10
    f = oracle.fields(L, 3.0, 5)
    b = oracle.basis(L)
    w = oracle.eigvalsh(oracle.dense_H(L, 1.0, f, b))
    # global spin flip: H(-h) isospectral (so the sign of the field term is immaterial)
    assert np.abs(oracle.eigvalsh(oracle.dense_H(L, 1.0, -f, b)) - w).max() < 1e-12
    # reflection i -> L-1-i with reversed fields
    assert np.abs(oracle.eigvalsh(oracle.dense_H(L, 1.0, f[::-1].copy(), b)) - w).max() < 1e-12
    # translation by one site with cyclically shifted fields
    assert np.abs(oracle.eigvalsh(oracle.dense_H(L, 1.0, np.roll(f, 1), b)) - w).max() < 1e-12


def test_translation_by_half_keeps_observables():
    L = 10
    f = oracle.fields(L, 2.0, 9)
    a = oracle.solve(L, 2.0, 9, 0.5, 6, fields_in=f)
    t = oracle.solve(L, 2.0, 9, 0.5, 6, fields_in=np.roll(f, L // 2))
    assert np.abs(a["evals"] - t["evals"]).max() < 1e-12
    assert np.abs(a["s1"] - t["s1"]).max() < 1e-9
    assert np.abs(a["se"] - t["se"]).max() < 1e-9   # cut at L/2 maps to itself
    fl = oracle.solve(L, 2.0, 9, 0.5, 6, fields_in=-f)
    assert np.abs(a["se"] - fl["se"]).max() < 1e-9 and np.abs(a["s1"] - fl["s1"]).max() < 1e-9


# -------------------------------------------------------------- observables

@pytest.mark.parametrize("L", [8, 10, 12])
def test_uniform_state_entropies(L):
    b = oracle.basis(L)
    psi = np.ones(b.size)
    assert abs(oracle.participation_entropy(psi, 1.0) - math.log(b.size)) < 1e-12
    assert abs(oracle.participation_entropy(psi, 2.0) - math.log(b.size)) < 1e-12
    wk = np.array([math.comb(L // 2, k) ** 2 for k in range(L // 2 + 1)]) / math.comb(L, L // 2)
    se = -np.sum(wk * np.log(wk))
    assert abs(oracle.entanglement_entropy(L, psi, b) - se) < 1e-12
    ref = {8: 1.13807, 10: 1.23587, 12: 1.31806}[L]
    assert abs(se - ref) < 1e-5


def test_singlet_products_entanglement():
    # s singlets straddling the cut (pairs (i, i + L/2)): S_E = s ln 2
    L = 8
    b = oracle.basis(L)
    la = L // 2

    def singlet_state(pairs, others_up):
        psi = np.zeros(b.size)
        for k, s in enumerate(b):
            s = int(s)
            amp = 1.0
            ok = True
            for (i, j) in pairs:
                bi, bj = (s >> i) & 1, (s >> j) & 1
                if bi == bj:
                    ok = False
                    break
                amp *= 1 / math.sqrt(2) if bi == 1 else -1 / math.sqrt(2)
            for (i, v) in others_up:
                if ((s >> i) & 1) != v:
                    ok = False
            if ok:
                psi[k] = amp
        return psi

    for s_count in range(0, la + 1):
        pairs = [(i, i + la) for i in range(s_count)]
        rest = [i for i in range(L) if all(i not in p for p in pairs)]
        # fill the remaining sites with one up in A, one down in B, etc. (S^z = 0 overall)
        others = []
        ra = [i for i in rest if i < la]
        rb = [i for i in rest if i >= la]
        for i in ra:
            others.append((i, 1))
        for i in rb:
            others.append((i, 0))
        psi = singlet_state(pairs, others)
        assert abs(np.linalg.norm(psi) - 1) < 1e-12
        assert abs(oracle.entanglement_entropy(L, psi, b) - s_count * math.log(2)) < 1e-12


def test_entanglement_vs_numpy_svd():
    L = 10
    out = oracle.solve(L, 1.0, 4, 0.5, 4)
    b = oracle.basis(L)
    la = L // 2
    for j in range(4):
        M = np.zeros((2 ** (L - la), 2 ** la))
        for k, s in enumerate(b):
            M[int(s) >> la, int(s) & (2 ** la - 1)] = out["evecs"][k, j]
        sv = np.linalg.svd(M, compute_uv=False) ** 2
        sv = sv[sv > 0]
        assert abs(-np.sum(sv * np.log(sv)) - out["se"][j]) < 1e-11


def test_basis_state_observables():
    L = 10
    b = oracle.basis(L)
    psi = np.zeros(b.size)
    psi[17] = 1.0
    assert oracle.participation_entropy(psi, 1.0) == 0.0
    assert abs(oracle.participation_entropy(psi, 2.0)) < 1e-15
    assert abs(oracle.entanglement_entropy(L, psi, b)) < 1e-14
    assert abs(oracle.bipartite_fluct(L, psi, b)) < 1e-15
    assert abs(oracle.dynamical_fraction(L, psi, b)) < 1e-14
    assert oracle.kl_divergence(psi, psi) == 0.0


def test_fluctuations_uniform_state_closed_form():
    # uniform sector state: S^z_A = n_A - L/4 with n_A hypergeometric(L, L/2, L/2):
    # Var = (L/2)(1/2)(1/2)(L - L/2)/(L - 1)
    L = 12
    b = oracle.basis(L)
    v = oracle.bipartite_fluct(L, np.ones(b.size), b)
    n, K, N = L // 2, L // 2, L
    var = n * (K / N) * (1 - K / N) * (N - n) / (N - 1)
    assert abs(v - var) < 1e-12


def test_kl_two_state_closed_form():
    # p = (1/2, 1/2, 0...), q = (1/4, 3/4, 0...): KL = 1/2 ln 2 + 1/2 ln(2/3)
    psi = np.zeros(6); psi[:2] = math.sqrt(0.5)
    phi = np.zeros(6); phi[0] = 0.5; phi[1] = math.sqrt(0.75)
    exp = 0.5 * math.log(0.5 / 0.25) + 0.5 * math.log(0.5 / 0.75)
    assert abs(oracle.kl_divergence(psi, phi) - exp) < 1e-15
    phi2 = np.zeros(6); phi2[0] = 1.0
    assert oracle.kl_divergence(psi, phi2) == math.inf


def test_dynamical_fraction_pins_the_wave_vector():
    # Supplementary "Dynamical spin fraction": M = sum_j S^z_j exp(2 pi i j / L),
    # site j = bit j-1.  L = 4, psi = 1/2 |word 3> + sqrt(3)/2 |word 5>:
    # word 3 (sites 1, 2 up) has m = (i - 1 - (-i) - 1) / 2 = i - 1, word 5
    # (sites 1, 3 up) has m = (i + 1 - i - 1) / 2 = 0, so <M> = (i - 1) / 4,
    # |<M>|^2 = 1/8, <|M|^2> = |i - 1|^2 / 4 = 1/2 and f = 1 - 1/4 = 3/4.
    # Another wave-vector changes it (pi / L gives 0.17, 4 pi / L gives 1/4).
    L = 4
    b = oracle.basis(L)
    psi = np.zeros(b.size)
    psi[oracle.rank(b, 3)] = 0.5
    psi[oracle.rank(b, 5)] = math.sqrt(3.0) / 2.0
    assert abs(oracle.dynamical_fraction(L, psi, b) - 0.75) < 1e-14


def test_dynamical_fraction_two_configurations():
    # equal-weight superposition of a Neel state and its flip: <M> = 0, f = 1
    L = 8
    b = oracle.basis(L)
    neel = sum(1 << i for i in range(0, L, 2))
    psi = np.zeros(b.size)
    psi[oracle.rank(b, neel)] = 1
    psi[oracle.rank(b, (2 ** L - 1) ^ neel)] = 1
    assert abs(oracle.dynamical_fraction(L, psi, b) - 1.0) < 1e-14


def test_gap_ratio_hand_example_and_degenerate():
    r, m = oracle.gap_ratios(np.array([0.0, 1.0, 3.0, 4.0]))
    assert np.allclose(r, [0.5, 0.5]) and abs(m - 0.5) < 1e-15
    r, _ = oracle.gap_ratios(np.array([1.0, 1.0, 1.0, 2.0]))
    assert math.isnan(r[0]) and r[1] == 0.0


def test_gap_ratio_poisson_limit_printed_in_paper():
    # item (i): r_Poisson = 2 ln 2 - 1 ~ 0.3863 for uncorrelated levels
    rng = np.random.default_rng(0)
    E = np.sort(rng.random(400000))
    _, m = oracle.gap_ratios(E)
    assert abs(m - (2 * math.log(2) - 1)) < 3e-3


def test_gap_ratio_goe_limit_printed_in_paper():
    # item (i): r_GOE = 0.5307(1); bulk of 300x300 GOE matrices
    rng = np.random.default_rng(1)
    vals = []
    for _ in range(40):
        A = rng.standard_normal((300, 300))
        w = oracle.eigvalsh((A + A.T) / 2)
        r, _ = oracle.gap_ratios(w[75:225])
        vals.append(r)
    m = np.mean(np.concatenate(vals))
    assert abs(m - 0.5307) < 0.01


def test_residual_and_rayleigh_helpers():
    L = 10
    out = oracle.solve(L, 3.0, 2, 0.3, 5)
    for j in range(5):
        psi = out["evecs"][:, j]
        assert oracle.residual(L, 1.0, out["fields"], psi, out["evals"][j]) < 1e-12
        assert abs(oracle.rayleigh(L, 1.0, out["fields"], psi) - out["evals"][j]) < 1e-12
    H = oracle.dense_H(L, 1.0, out["fields"])
    x = np.random.default_rng(0).standard_normal(H.shape[0])
    assert np.abs(oracle.apply_H(L, 1.0, out["fields"], x) - H @ x).max() < 1e-12


def _fake_target(evals, emin, emax, r, s1, s2, se, fluct, dynfrac, kl):
    return dict(evals=np.array(evals, float), emin=emin, emax=emax, r=np.array(r, float),
                s1=np.array(s1, float), s2=np.array(s2, float), se=np.array(se, float),
                fluct=np.array(fluct, float), dynfrac=np.array(dynfrac, float),
                kl=np.array(kl, float))


def test_realization_bins_hand_example():
    # averages over the eigenstates of one sample ("Numerical method" section):
    # r and KL average only their finite values; energy density (E - Emin)/(Emax - Emin)
    out = _fake_target([-1.0, 0.0, 1.0], -2.0, 2.0, [0.4],
                       [1.0, 2.0, 3.0], [0.5, 1.0, 1.5], [1.0, 2.0, 4.0], [0.1, 0.2, 0.3],
                       [0.9, 0.6, 0.3], [math.inf, 1.0])
    b = oracle.realization_bins(out)
    assert b[0] == pytest.approx(0.4)
    assert b[1] == pytest.approx(2.0) and b[2] == pytest.approx(1.0)
    assert b[3] == pytest.approx(7.0 / 3.0)
    assert b[4] == pytest.approx(21.0 / 3.0)               # (1 + 4 + 16) / 3
    assert b[5] == pytest.approx(0.2) and b[6] == pytest.approx(0.6)
    assert b[7] == pytest.approx(1.0)                      # the infinite KL is left out
    assert b[8] == pytest.approx(0.5)                      # (0.25 + 0.5 + 0.75) / 3
    assert b[9] == 3
    out4 = _fake_target([-1.0, 0.0, 0.5, 1.0], -2.0, 2.0, [0.5, math.nan], [0] * 4, [0] * 4,
                        [0] * 4, [0] * 4, [0] * 4, [0] * 3)
    assert oracle.realization_bins(out4)[0] == pytest.approx(0.5)   # a NaN ratio is skipped


def test_disorder_average_hand_example():
    # two samples with S_E = {1, 3} and {3, 5}: pooled states {1, 3, 3, 5} have
    # mean 3 and variance 2, so sigma_E = sqrt(2); r bins 1..4 -> SEM sqrt(5/12)
    t1 = _fake_target([0.0, 1.0], 0.0, 1.0, [], [0, 0], [0, 0], [1.0, 3.0], [0, 0], [0, 0], [0.0])
    t2 = _fake_target([0.0, 1.0], 0.0, 1.0, [], [0, 0], [0, 0], [3.0, 5.0], [0, 0], [0, 0], [0.0])
    B = np.array([oracle.realization_bins(t1), oracle.realization_bins(t2)])
    avg = oracle.disorder_average(B)
    assert avg["mean"][3] == pytest.approx(3.0)
    assert avg["sigma_e"] == pytest.approx(math.sqrt(2.0))
    assert avg["sem"][3] == pytest.approx(1.0)             # bins 2 and 4: sqrt(2 / 2)
    assert math.isnan(avg["mean"][0])                      # nev = 2: no gap ratio
    R = np.zeros((4, len(oracle.BIN_NAMES)))
    R[:, 0] = [1.0, 2.0, 3.0, 4.0]
    R[2, 1] = math.nan                                     # a missing bin is skipped
    avg = oracle.disorder_average(R)
    assert avg["mean"][0] == pytest.approx(2.5)
    assert avg["sem"][0] == pytest.approx(math.sqrt(5.0 / 12.0))
    assert avg["mean"][1] == 0.0 and avg["sem"][1] == 0.0
    one = oracle.disorder_average(R[:1])
    assert math.isnan(one["sem"][0])                       # one sample: no error bar


# ------------------------------------------- odd L: the S^z = +1/2 sector

@pytest.mark.parametrize("L", [3, 5, 7, 9, 11, 13, 15])
def test_odd_sector_dimension_and_order(L):
    b = oracle.basis(L)
    nup = (L + 1) // 2
    assert oracle.sector_nup(L) == nup
    assert b.size == math.comb(L, nup)
    assert np.all(np.diff(b.astype(np.int64)) > 0)
    assert all(bin(int(s)).count("1") == nup for s in b[:: max(1, b.size // 97)])


def test_odd_sector_dimensions_of_the_paper_sizes():
    # the paper's odd chains 15, 17, 19 (and 21): C(L, (L+1)/2)
    assert [oracle.sector_dim(L) for L in (15, 17, 19, 21)] == [6435, 24310, 92378, 352716]


@pytest.mark.parametrize("L", [3, 5, 7, 9])
def test_odd_sector_block_equals_bruteforce(L):
    f = oracle.fields(L, 2.0, 13)
    Hf = _full_H(L, 1.0, f)
    assert np.abs(Hf.imag).max() < 1e-14
    Hf = Hf.real
    b = oracle.basis(L)
    Hs = oracle.dense_H(L, 1.0, f, b)
    assert np.abs(Hf[np.ix_(b, b)] - Hs).max() < 1e-14
    # the block is S^z = +1/2: <S^z_tot> = 1/2 on every basis state
    assert all(bin(int(s)).count("1") - L / 2 == 0.5 for s in b)
    wf = np.linalg.eigvalsh(Hf)
    for lam in oracle.eigvalsh(Hs):
        assert np.min(np.abs(wf - lam)) < 1e-12


@pytest.mark.parametrize("L", [5, 7, 9, 11])
@pytest.mark.parametrize("J", [1.0, 0.6])
def test_odd_trace_closed_form(L, J):
    # S^z = 1/2 on a ring of odd L: a bond is parallel with probability
    # (L-1)/(2L), so each bond contributes -J/(4L) on average; site i is up in
    # a fraction (L+1)/(2L) of the states, so sum_i h_i <S^z_i> = sum h / (2L)
    f = oracle.fields(L, 2.5, 100 + L)
    H = oracle.dense_H(L, J, f)
    dim = math.comb(L, (L + 1) // 2)
    tr = -J * dim / 4 + dim * np.sum(f) / (2 * L)
    assert abs(np.trace(H) - tr) < 1e-10 * dim
    assert abs(oracle.eigvalsh(H).sum() - tr) < 1e-9 * dim


def test_odd_entanglement_vs_numpy_svd():
    # A = sites 1..(L-1)/2 (low bits), B one site larger: rectangular blocks
    L = 9
    out = oracle.solve(L, 1.0, 4, 0.5, 4)
    b = oracle.basis(L)
    la = L // 2
    for j in range(4):
        M = np.zeros((2 ** (L - la), 2 ** la))
        for k, s in enumerate(b):
            M[int(s) >> la, int(s) & (2 ** la - 1)] = out["evecs"][k, j]
        sv = np.linalg.svd(M, compute_uv=False) ** 2
        sv = sv[sv > 0]
        assert abs(-np.sum(sv * np.log(sv)) - out["se"][j]) < 1e-11
        # S^z_A fluctuation: sites 1..la, B carries the extra half
        p = out["evecs"][:, j] ** 2
        sza = np.array([bin(int(s) & (2 ** la - 1)).count("1") - la / 2 for s in b])
        assert abs(p @ sza ** 2 - (p @ sza) ** 2 - out["fluct"][j]) < 1e-12
