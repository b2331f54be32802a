"""Pins for the CPU oracle: each check comes from the paper or from mathematics,
never from the oracle itself (CPU only)."""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np
import pytest

import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rnd(seed, shape, cplx=False):
    g = np.random.default_rng(seed)
    a = g.standard_normal(shape)
    if cplx:
        a = a + 1j * g.standard_normal(shape)
    return a


def skew(a):
    return 0.5 * (a - np.swapaxes(a, -1, -2))


# ----------------------------------------------------------------------------
# Determinant, log|det|, phase, inverse
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_det_matches_leibniz(oracle, n, cplx):
    a = rnd(10 + n, (n, n), cplx)
    ref = brute.leibniz_det(a.tolist())
    got = oracle.det(a)
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("seed", range(6))
def test_det_exact_integer(oracle, seed):
    g = np.random.default_rng(seed)
    n = 3 + seed
    a = g.integers(-5, 6, size=(n, n)).astype(float)
    ref = brute.exact_det(a.astype(int).tolist())
    got = oracle.det(a)
    assert abs(got - float(ref)) <= 1e-9 * max(1.0, abs(float(ref)))


def test_det_of_permutation_matrices_is_their_sign(oracle):
    g = np.random.default_rng(3)
    for n in (2, 5, 9, 16):
        for _ in range(5):
            p = g.permutation(n)
            a = np.zeros((n, n))
            a[np.arange(n), p] = 1.0
            la, ph, inv = oracle.slogdet(a)
            assert la == 0.0
            assert ph == brute.perm_sign(p)
            assert np.array_equal(inv, a.T)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [7, 32, 128, 256])
def test_slogdet_and_inverse_vs_lapack(oracle, n, cplx):
    a = rnd(100 + n, (3, n, n), cplx)
    la, ph, inv = oracle.slogdet(a)
    sref, lref = np.linalg.slogdet(a)
    np.testing.assert_allclose(la, lref, rtol=0, atol=1e-9 * n)
    np.testing.assert_allclose(ph, sref, rtol=0, atol=1e-9 * n)
    iref = np.linalg.inv(a)
    err = np.linalg.norm(inv - iref, axis=(1, 2)) / np.linalg.norm(iref, axis=(1, 2))
    cond = np.linalg.cond(a)
    assert np.all(err <= 1e-14 * n * cond)
    resid = np.linalg.norm(a @ inv - np.eye(n), axis=(1, 2))
    assert np.all(resid <= 1e-14 * n * cond)


def test_singular_matrix_flags(oracle):
    a = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [0.0, 1.0, 5.0]])
    la, ph, inv = oracle.slogdet(a)
    assert la == -np.inf and ph == 0.0 and np.isnan(inv).all()


def test_pivot_tie_goes_to_lowest_row(oracle):
    # Equal-magnitude candidates: the determinant is unique whatever the pivot,
    # the sign bookkeeping must still be right.
    a = np.array([[1.0, 1.0, 0.0], [-1.0, 1.0, 1.0], [1.0, 0.0, 1.0]])
    assert oracle.det(a) == pytest.approx(brute.leibniz_det(a.tolist()), abs=1e-15)


# ----------------------------------------------------------------------------
# Pfaffian (Appendix A)
# ----------------------------------------------------------------------------
def _golden_closed_forms():
    rows = []
    with open(os.path.join(GOLDEN, "pf_closed_forms.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            tok = line.split()
            rows.append((tok[0], [float(x) for x in tok[1:-1]], float(tok[-1])))
    return rows


@pytest.mark.parametrize("kind,vals,expected", _golden_closed_forms())
def test_pf_closed_forms_golden(oracle, kind, vals, expected):
    if kind == "2x2":
        a = np.array([[0.0, vals[0]], [-vals[0], 0.0]])
    else:
        a_, b_, c_, d_, e_, f_ = vals
        a = np.array([[0, a_, b_, c_], [-a_, 0, d_, e_], [-b_, -d_, 0, f_], [-c_, -e_, -f_, 0]], float)
    # the oracle returns exp(log|pf|) * phase: exact up to the rounding of exp/log
    assert abs(oracle.pf(a) - expected) <= 4e-15 * max(1.0, abs(expected))


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [2, 4, 6, 8, 10])
def test_pf_matches_perfect_matching_sum(oracle, n, cplx):
    a = skew(rnd(200 + n, (n, n), cplx))
    ref = brute.matching_pf(a.tolist())
    got = oracle.pf(a)
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))


def test_pf_exact_integer_matching_sum(oracle):
    g = np.random.default_rng(7)
    for n in (4, 6, 8):
        m = g.integers(-4, 5, size=(n, n))
        a = np.triu(m, 1)
        a = a - a.T
        ref = brute.matching_pf(a.astype(int).tolist())
        assert abs(oracle.pf(a.astype(float)) - ref) <= 1e-9 * max(1, abs(ref))


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [16, 64, 256])
def test_pf_squared_is_det(oracle, n, cplx):
    a = skew(rnd(300 + n, (2, n, n), cplx))
    la, ph = oracle.slogpf(a)
    sref, lref = np.linalg.slogdet(a)
    np.testing.assert_allclose(2 * la, lref, rtol=0, atol=1e-9 * n)
    np.testing.assert_allclose(ph ** 2, sref, rtol=0, atol=1e-9 * n)


@pytest.mark.parametrize("cplx", [False, True])
def test_pf_congruence(oracle, cplx):
    # pf(B A B^T) = det(B) pf(A)  (Appendix A, Eq. pf->det_pf)
    for n in (4, 10, 40):
        a = skew(rnd(400 + n, (n, n), cplx))
        b = rnd(500 + n, (n, n), cplx)
        lhs = oracle.pf(b @ a @ b.T)
        rhs = np.linalg.det(b) * oracle.pf(a)
        assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 7])
def test_pf_block_offdiagonal(oracle, m):
    # pf [[0, X], [-X^T, 0]] = (-1)^{m(m-1)/2} det X   (Appendix A, Eq. pf_offdiagonal)
    x = rnd(600 + m, (m, m))
    a = np.block([[np.zeros((m, m)), x], [-x.T, np.zeros((m, m))]])
    ref = (-1) ** (m * (m - 1) // 2) * np.linalg.det(x)
    assert abs(oracle.pf(a) - ref) <= 1e-12 * max(1, abs(ref))


def test_pf_skew_identity(oracle):
    # pf J = (-1)^{k(k-1)/2} for J = [[0, 1], [-1, 0]] in k x k blocks (Sec. III.A)
    for k in range(1, 7):
        j = np.block([[np.zeros((k, k)), np.eye(k)], [-np.eye(k), np.zeros((k, k))]])
        assert oracle.pf(j) == (-1) ** (k * (k - 1) // 2)


def test_pf_block_diagonal(oracle):
    # pf diag(A, A') = pf(A) pf(A')   (Appendix A, Eq. pf_diagonal)
    a = skew(rnd(700, (6, 6), True))
    b = skew(rnd(701, (8, 8), True))
    z = np.zeros((6, 8))
    big = np.block([[a, z], [z.T, b]])
    assert abs(oracle.pf(big) - oracle.pf(a) * oracle.pf(b)) <= 1e-12 * abs(oracle.pf(big))


def test_pf_odd_dimension_is_zero(oracle):
    la, ph = oracle.slogpf(skew(rnd(8, (5, 5))))
    assert la == -np.inf and ph == 0.0


def test_pf_zero_column(oracle):
    a = skew(rnd(9, (6, 6)))
    a[2, :] = 0.0
    a[:, 2] = 0.0
    la, ph = oracle.slogpf(a)
    assert la == -np.inf and ph == 0.0


def test_pf_block_schur(oracle):
    # pf [[M, Q], [-Q^T, N]] = pf(M) pf(N + Q^T M^-1 Q)   (Appendix A, Eq. pf_block)
    g = np.random.default_rng(11)
    m = skew(g.standard_normal((4, 4)))
    nn = skew(g.standard_normal((6, 6)))
    q = g.standard_normal((4, 6))
    big = np.block([[m, q], [-q.T, nn]])
    rhs = oracle.pf(m) * oracle.pf(nn + q.T @ np.linalg.inv(m) @ q)
    assert abs(oracle.pf(big) - rhs) <= 1e-11 * abs(rhs)


# ----------------------------------------------------------------------------
# Ratios: the low-rank identities themselves, and telescoping
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_determinant_lemma(oracle, k, cplx):
    # det(A + v u^T) / det(A) = det(1 + u^T A^-1 v)   (Sec. II.A, Eqs. det_ratio, det_R)
    n = 9
    a = rnd(800 + k, (n, n), cplx)
    u = rnd(810 + k, (n, k), cplx)
    v = rnd(820 + k, (n, k), cplx)
    la0, ph0, _ = oracle.slogdet(a)
    la1, ph1, _ = oracle.slogdet(a + v @ u.T)
    r = oracle.ratio(la1, ph1, la0, ph0)
    ref = np.linalg.det(np.eye(k) + u.T @ np.linalg.inv(a) @ v)
    assert abs(r - ref) <= 1e-11 * abs(ref)


@pytest.mark.parametrize("cplx", [False, True])
def test_pf_low_rank_identity(oracle, cplx):
    # pf(A - u J u^T)/pf(A) = pf(J + u^T A^-1 u)/pf(J)   (Sec. III.A, Eqs. pf_ratio, pf_R)
    for k in (1, 2):
        n = 10
        a = skew(rnd(900 + k, (n, n), cplx))
        u = rnd(910 + k, (n, 2 * k), cplx)
        j = np.block([[np.zeros((k, k)), np.eye(k)], [-np.eye(k), np.zeros((k, k))]])
        la0, ph0 = oracle.slogpf(a)
        la1, ph1 = oracle.slogpf(a - u @ j @ u.T)
        r = oracle.ratio(la1, ph1, la0, ph0)
        rr = j + u.T @ np.linalg.inv(a) @ u
        ref = brute.matching_pf(skew(rr).tolist()) / (-1) ** (k * (k - 1) // 2)
        assert abs(r - ref) <= 1e-10 * abs(ref)


def test_slater_hop_special_case_and_telescoping(oracle):
    # Single hop of electron i from site s to s': r = Phi[s'] . A^-1[:, i]
    # (rank-1 row update, Sec. II.B); the product of ratios telescopes.
    from paper_2602_05255_amd import inputs as gen
    g = gen.generator(5)
    L, n, W = 24, 10, 4
    phi = gen.normal(g, (L, n))
    occ, emp = gen.occupancy(g, W, L, n)
    chain = oracle.DetChain(phi, occ, emp)
    la_start = chain.logabs.copy()
    ph_start = chain.phase.copy()
    logprod = np.zeros(W)
    sgn = np.ones(W)
    for t in range(30):
        k, elec, slot = gen.hop_draws(g, W, n, L - n, (1,), 1)
        inv_before = chain.inv.copy()
        occ_before = chain.book.occ.copy()
        emp_before = chain.book.empty.copy()
        r = chain.propose(k, elec, slot)
        for w in range(W):
            i = elec[w, 0]
            s_new = emp_before[w, slot[w, 0]]
            ref = phi[s_new] @ np.linalg.inv(phi[occ_before[w]])[:, i]
            assert abs(r[w] - ref) <= 1e-10 * abs(ref)
            assert abs(r[w] - phi[s_new] @ inv_before[w][:, i]) <= 1e-10 * abs(ref)
        chain.accept(k, elec, slot, np.ones(W, bool))
        logprod += np.log(np.abs(r))
        sgn *= np.sign(r)
    sref, lref = np.linalg.slogdet(phi[chain.book.occ])
    np.testing.assert_allclose(logprod, lref - la_start, atol=1e-9)
    np.testing.assert_array_equal(sgn, sref * ph_start)


def test_pf_hop_special_case(oracle):
    # Hop of electron i in the Pfaffian state: row i += x, column i -= x with
    # x_j = F[s', occ_j] - F[s, occ_j]; r = pf R_1 = 1 + x . A^-1[:, i]  (Eqs. pf_rank2, pf_R)
    from paper_2602_05255_amd import inputs as gen
    g = gen.generator(6)
    L, n, W = 20, 8, 3
    f = gen.skew_from(gen.normal(g, (L, L), True))
    occ, emp = gen.occupancy(g, W, L, n)
    chain = oracle.PfChain(f, occ, emp)
    for t in range(10):
        k, elec, slot = gen.hop_draws(g, W, n, L - n, (1,), 1)
        occ_b = chain.book.occ.copy()
        emp_b = chain.book.empty.copy()
        inv_b = chain.inv.copy()
        r = chain.propose(k, elec, slot)
        for w in range(W):
            i = elec[w, 0]
            s, s2 = occ_b[w, i], emp_b[w, slot[w, 0]]
            x = f[s2, occ_b[w]] - f[s, occ_b[w]]
            x[i] = 0.0
            ref = 1.0 + x @ inv_b[w][:, i]
            assert abs(r[w] - ref) <= 1e-10 * abs(ref)
            a_old = f[np.ix_(occ_b[w], occ_b[w])]
            e = np.zeros(n)
            e[i] = 1
            a_new = a_old + np.outer(e, x) - np.outer(x, e)
            occ_new = occ_b[w].copy()
            occ_new[i] = s2
            np.testing.assert_allclose(a_new, f[np.ix_(occ_new, occ_new)], atol=1e-14)
        chain.accept(k, elec, slot, np.ones(W, bool))
    # pf inverse stays exactly skew
    assert np.array_equal(chain.inv, -np.swapaxes(chain.inv, -1, -2))


# ----------------------------------------------------------------------------
# Delayed recurrences in exact arithmetic equal full recompute (Sec. II.C, III.C)
# ----------------------------------------------------------------------------
def _int_matrix(g, n, lo=-3, hi=4):
    while True:
        a = g.integers(lo, hi, size=(n, n))
        if brute.exact_det(a.tolist()) != 0:
            return brute.frac_matrix(a.tolist())


def test_delayed_det_recurrences_exact():
    """Eqs. det_a, det_b, delayed_Ainv and the R_tau / a_tau / b_tau recurrences, with
    the delay counter read as: a step at slot tau uses slots 1..tau-1 (exact rationals)."""
    g = np.random.default_rng(21)
    n, T = 6, 4
    a = _int_matrix(g, n)
    a0inv = brute.exact_inverse(a)
    slots = []
    cur = [row[:] for row in a]
    for step in range(9):
        tau = len(slots)
        k = 1 + step % 2
        rows = list(g.choice(n, size=k, replace=False))
        v = [[Fraction(int(i == rows[c])) for c in range(k)] for i in range(n)]
        u = brute.frac_matrix(g.integers(-2, 3, size=(n, k)).tolist())
        ut, vt = brute.transpose(u), brute.transpose(v)
        # R_tau = 1 + u^T A0^-1 v - sum_t (u^T a_t)(b_t^T v)
        r = brute.add(brute.eye(k), brute.matmul(brute.matmul(ut, a0inv), v))
        for at, bt in slots:
            r = brute.sub(r, brute.matmul(brute.matmul(ut, at), brute.matmul(brute.transpose(bt), v)))
        if brute.exact_det(r) == 0:
            continue
        new = brute.add(cur, brute.matmul(v, ut))
        ratio = brute.exact_det(new) / brute.exact_det(cur)
        assert brute.exact_det(r) == ratio
        rinv = brute.exact_inverse(r)
        # a_tau = A0^-1 v - sum a_t (b_t^T v);  b_tau = [A0^-T u - sum b_t (a_t^T u)] R^-T
        at_new = brute.matmul(a0inv, v)
        bt_new = brute.matmul(brute.transpose(a0inv), u)
        for at, bt in slots:
            at_new = brute.sub(at_new, brute.matmul(at, brute.matmul(brute.transpose(bt), v)))
            bt_new = brute.sub(bt_new, brute.matmul(bt, brute.matmul(brute.transpose(at), u)))
        bt_new = brute.matmul(bt_new, brute.transpose(rinv))
        slots.append((at_new, bt_new))
        cur = new
        recon = a0inv
        for at, bt in slots:
            recon = brute.sub(recon, brute.matmul(at, brute.transpose(bt)))
        assert recon == brute.exact_inverse(cur)
        if len(slots) == T:                   # flush: A_tau^-1 becomes the new A0^-1
            a0inv, slots = recon, []


def test_delayed_pf_recurrences_exact():
    """Eqs. pf_a, pf_delayed_Ainv and the R_tau / a_tau recurrences (a_tau uses u_tau:
    the u_t inside the first term of the a_tau formula is read as u_tau), exact rationals."""
    g = np.random.default_rng(22)
    n, T = 6, 3
    while True:
        m = g.integers(-3, 4, size=(n, n))
        m = np.triu(m, 1)
        m = m - m.T
        if brute.exact_det(m.tolist()) != 0:
            break
    a = brute.frac_matrix(m.tolist())
    a0inv = brute.exact_inverse(a)
    j2 = [[Fraction(0), Fraction(1)], [Fraction(-1), Fraction(0)]]
    slots = []
    cur = [row[:] for row in a]
    for step in range(7):
        i = int(g.integers(0, n))
        x = [Fraction(int(t)) for t in g.integers(-2, 3, size=n)]
        x[i] = Fraction(0)
        u = [[x[q], Fraction(int(q == i))] for q in range(n)]      # u = (x, e_i)
        ut = brute.transpose(u)
        r = brute.add(j2, brute.matmul(brute.matmul(ut, a0inv), u))
        for at, rt in slots:
            uta = brute.matmul(ut, at)
            r = brute.add(r, brute.matmul(brute.matmul(uta, rt), brute.transpose(uta)))
        if r[0][1] == 0:
            continue
        new = brute.sub(cur, brute.matmul(brute.matmul(u, j2), ut))
        assert brute.matching_pf(new) / brute.matching_pf(cur) == r[0][1]   # pf R / pf J, pf J = 1
        rinv = brute.exact_inverse(r)
        at_new = brute.matmul(a0inv, u)
        for at, rt in slots:
            at_new = brute.add(at_new, brute.matmul(brute.matmul(at, rt),
                                                    brute.transpose(brute.matmul(ut, at))))
        slots.append((at_new, rinv))
        cur = new
        recon = a0inv
        for at, rt in slots:
            recon = brute.add(recon, brute.matmul(brute.matmul(at, rt), brute.transpose(at)))
        assert recon == brute.exact_inverse(cur)
        if len(slots) == T:
            a0inv, slots = recon, []


def test_padded_rank_is_exact():
    """Padding a rank-k update to k_max with zero u-columns (repeated valid row index)
    leaves the ratio and the Woodbury update unchanged (reading of the rank draws)."""
    g = np.random.default_rng(23)
    n = 7
    a = _int_matrix(g, n)
    ainv = brute.exact_inverse(a)
    rows = [2, 5]
    u = brute.frac_matrix(g.integers(-2, 3, size=(n, 2)).tolist())
    up = [r + [Fraction(0), Fraction(0)] for r in u]
    rows_p = rows + [rows[0], rows[0]]
    for uu, rr in ((u, rows), (up, rows_p)):
        k = len(rr)
        v = [[Fraction(int(i == rr[c])) for c in range(k)] for i in range(n)]
        r = brute.add(brute.eye(k), brute.matmul(brute.matmul(brute.transpose(uu), ainv), v))
        if uu is u:
            ref_det = brute.exact_det(r)
            upd = brute.sub(ainv, brute.matmul(brute.matmul(brute.matmul(ainv, v), brute.exact_inverse(r)),
                                               brute.matmul(brute.transpose(uu), ainv)))
        else:
            assert brute.exact_det(r) == ref_det
            upd2 = brute.sub(ainv, brute.matmul(brute.matmul(brute.matmul(ainv, v), brute.exact_inverse(r)),
                                                brute.matmul(brute.transpose(uu), ainv)))
            assert upd2 == upd


# ----------------------------------------------------------------------------
# Gradients (Appendix A, Eq. pf_grad; log det)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("cplx", [False, True])
def test_lowrank_logdet_gradients_fd(oracle, cplx):
    g = np.random.default_rng(31)
    L, n, r, S = 12, 6, 2, 2
    phi = g.standard_normal((L, n)) + (1j * g.standard_normal((L, n)) if cplx else 0)
    occ = np.stack([np.sort(g.permutation(L)[:n]) for _ in range(S)])
    b = 0.3 * (g.standard_normal((S, n, r)) + (1j * g.standard_normal((S, n, r)) if cplx else 0))
    c = 0.3 * (g.standard_normal((S, n, r)) + (1j * g.standard_normal((S, n, r)) if cplx else 0))
    la, ph, gm, gb, gc = oracle.lowrank_logdet_and_grads(phi, occ, b, c)

    def logdet(phi_, b_, c_):
        m = phi_[occ] + b_ @ np.swapaxes(c_, -1, -2)
        s, l = np.linalg.slogdet(m)
        return l + (np.log(s) if cplx else 0)   # holomorphic log det (real: log|det|)

    h = 1e-6
    # d/dPhi[site, col] = sum over electrons on that site of G[i, col]
    gphi = np.stack([oracle.scatter_rows(gm[s:s + 1], occ[s:s + 1], L) for s in range(S)])
    for (site, col) in [(occ[0, 1], 2), (occ[1, 3], 0), (occ[0, 5], 5)]:
        d = np.zeros_like(phi)
        d[site, col] = h
        fd = (logdet(phi + d, b, c) - logdet(phi - d, b, c)) / (2 * h)
        np.testing.assert_allclose(fd, gphi[:, site, col], atol=1e-7)
    for (i, q) in [(0, 0), (3, 1), (5, 1)]:
        d = np.zeros_like(b)
        d[:, i, q] = h
        fd = (logdet(phi, b + d, c) - logdet(phi, b - d, c)) / (2 * h)
        np.testing.assert_allclose(fd, gb[:, i, q], atol=1e-7)
        fd = (logdet(phi, b, c + d) - logdet(phi, b, c - d)) / (2 * h)
        np.testing.assert_allclose(fd, gc[:, i, q], atol=1e-7)


@pytest.mark.parametrize("cplx", [False, True])
def test_pf_gradient_formula_fd(oracle, cplx):
    # d pf(A')/dA_ij = (1/2) pf(A') (A'^-1)_ji with A' = (A - A^T)/2  (Appendix A, Eq. pf_grad)
    g = np.random.default_rng(41)
    n = 8
    a = g.standard_normal((n, n)) + (1j * g.standard_normal((n, n)) if cplx else 0)
    ap = skew(a)
    p0 = oracle.pf(ap)
    inv = oracle.skew_inverse(ap)
    h = 1e-6
    for (i, j) in [(0, 1), (2, 5), (7, 3), (4, 4)]:
        d = np.zeros_like(a)
        d[i, j] = h
        fd = (oracle.pf(skew(a + d)) - oracle.pf(skew(a - d))) / (2 * h)
        assert abs(fd - 0.5 * p0 * inv[j, i]) <= 1e-7 * max(1, abs(p0))


@pytest.mark.parametrize("cplx", [False, True])
def test_lowrank_logpf_gradients_fd(oracle, cplx):
    """log pf(F[occ][:, occ] - U J U^T) and its gradients with respect to U and to the
    pairing matrix F (through the gather, skew directions), by central differences of the
    Pfaffian itself, and the Pfaffian low-rank identity for the value (App. A, Eq.
    pf_low_rank: pf(A - U J U^T) = pf(A) pf(J + U^T A^-1 U) / pf(J), with J^-1 = -J)."""
    g = np.random.default_rng(51)
    L, n, k, S = 12, 6, 2, 2
    z = (lambda sh: g.standard_normal(sh) + 1j * g.standard_normal(sh)) if cplx else g.standard_normal
    f = skew(z((L, L)))
    occ = np.stack([np.sort(g.permutation(L)[:n]) for _ in range(S)])
    u = 0.4 * z((S, n, 2 * k))
    la, ph, gm, gu = oracle.lowrank_logpf_and_grads(f, occ, u)
    jm = oracle.skew_eye(k)
    a = oracle.pairing_matrices(f, occ)
    for s in range(S):
        # value by the low-rank identity, with brute-force perfect-matching Pfaffians
        pa = brute.matching_pf(a[s].tolist())
        pr = brute.matching_pf((jm + u[s].T @ np.linalg.inv(a[s]) @ u[s]).tolist())
        pj = (-1) ** (k * (k - 1) // 2)
        want = pa * pr / pj
        assert abs(ph[s] * np.exp(la[s]) - want) <= 1e-10 * abs(want)

    def logpf(f_, u_):
        m = oracle.pairing_matrices(f_, occ) - u_ @ jm @ np.swapaxes(u_, -1, -2)
        l_, p_ = oracle.slogpf(m)
        return l_ + (np.log(p_) if cplx else 0)     # holomorphic log pf (real: log|pf|)

    h = 1e-6
    for (i, q) in [(0, 0), (3, 1), (5, 3), (2, 2)]:
        d = np.zeros_like(u)
        d[:, i, q] = h
        fd = (logpf(f, u + d) - logpf(f, u - d)) / (2 * h)
        np.testing.assert_allclose(fd, gu[:, i, q], atol=1e-7)
    gf = np.stack([oracle.scatter_pairs(gm[s:s + 1], occ[s:s + 1], L) for s in range(S)])
    for (p_, q_) in [(occ[0, 1], occ[0, 4]), (occ[1, 0], occ[1, 5]), (occ[0, 2], occ[1, 3])]:
        d = np.zeros_like(f)
        d[p_, q_] = h
        d[q_, p_] = -h            # a skew direction keeps F skew
        fd = (logpf(f + d, u) - logpf(f - d, u)) / (2 * h)
        np.testing.assert_allclose(fd, gf[:, p_, q_] - gf[:, q_, p_], atol=1e-7)


# ----------------------------------------------------------------------------
# General update forms (Sec. II.B and III.B, "Matrix updates")
# ----------------------------------------------------------------------------
def test_det_general_update_forms_match_the_displayed_matrices(oracle):
    """The oracle's A_1 - A_0 for the displayed examples of Sec. II.B: rank-1 row, rank-1
    column, rank-2 row and the simultaneous row + column update (row 1 gains u, column 2
    gains v, the crossing gets u_2 + v_1)."""
    z = np.zeros((1, 4, 4))
    u = np.array([2.0, 3.0, 5.0, 7.0])
    v = np.array([11.0, 13.0, 17.0, 19.0])
    d = oracle.det_general_matrix(z, [[1]], [[u]], None, None)[0]
    want = np.zeros((4, 4))
    want[1] = u
    np.testing.assert_array_equal(d, want)
    d = oracle.det_general_matrix(z, None, None, [[2]], [[v]])[0]
    want = np.zeros((4, 4))
    want[:, 2] = v
    np.testing.assert_array_equal(d, want)
    u2 = np.array([[2.0, 3.0, 5.0, 7.0], [23.0, 29.0, 31.0, 37.0]])
    d = oracle.det_general_matrix(z, [[1, 3]], [u2], None, None)[0]
    want = np.zeros((4, 4))
    want[1], want[3] = u2[0], u2[1]
    np.testing.assert_array_equal(d, want)
    d = oracle.det_general_matrix(z, [[1]], [[u]], [[2]], [[v]])[0]
    want = np.array([[0, 0, 11, 0], [2, 3, 5 + 13, 7], [0, 0, 17, 0], [0, 0, 19, 0]], dtype=float)
    np.testing.assert_array_equal(d, want)


def test_pf_general_update_forms_match_the_displayed_matrices(oracle):
    """The oracle's A_1 - A_0 = -u J u^T for the displayed examples of Sec. III.B: 1 row
    and 1 column (u = (x, e_1)) and 2 rows and 2 columns (u = (x_0, x_1, e_1, e_3))."""
    z = np.zeros((1, 4, 4))
    x = np.array([2.0, 3.0, 5.0, 7.0])
    d = oracle.pf_general_matrix(z, [[1]], [[x]])[0]
    want = np.array([[0, -2, 0, 0], [2, 0, 5, 7], [0, -5, 0, 0], [0, -7, 0, 0]], dtype=float)
    np.testing.assert_array_equal(d, want)
    z6 = np.zeros((1, 6, 6))
    u0 = np.array([2.0, 3.0, 5.0, 7.0, 11.0, 13.0])
    u1 = np.array([17.0, 19.0, 23.0, 29.0, 31.0, 37.0])
    d = oracle.pf_general_matrix(z6, [[1, 3]], [[u0, u1]])[0]
    want = np.array([
        [0, -u0[0], 0, -u1[0], 0, 0],
        [u0[0], 0, u0[2], u0[3] - u1[1], u0[4], u0[5]],
        [0, -u0[2], 0, -u1[2], 0, 0],
        [u1[0], u1[1] - u0[3], u1[2], 0, u1[4], u1[5]],
        [0, -u0[4], 0, -u1[4], 0, 0],
        [0, -u0[5], 0, -u1[5], 0, 0]])
    np.testing.assert_array_equal(d, want)


def test_metropolis_rule(oracle):
    r = np.array([2.0, 0.5, -0.5, 0.0, np.nan, 1j])
    u = np.array([0.99, 0.24, 0.26, 0.0, 0.0, 0.5])
    np.testing.assert_array_equal(oracle.metropolis(r, u), [True, True, False, False, False, True])


def test_occupancy_hop_semantics(oracle):
    occ = np.array([[0, 2, 5]])
    emp = np.array([[1, 3, 4, 6]])
    book = oracle.Occupancy(occ, emp)
    k = np.array([2])
    elec = np.array([[0, 2]])
    slot = np.array([[3, 1]])
    np.testing.assert_array_equal(book.proposed(k, elec, slot), [[6, 2, 3]])
    book.commit(k, elec, slot, np.array([True]))
    np.testing.assert_array_equal(book.occ, [[6, 2, 3]])
    np.testing.assert_array_equal(book.empty, [[1, 5, 4, 0]])


@pytest.mark.parametrize("kind", ["det", "pf"])
def test_chain_partial_accept_mask(oracle, kind):
    """A step with a mixed accept mask: every accepted walker's state is the inverse and
    log-magnitude of the matrix gathered at its new occupancy (checked by the residual
    A_new A^-1 = I and by LAPACK's slogdet, not by the oracle's own routines), and every
    rejected walker's state is bitwise unchanged (Sec. II.A / III.A: a rejected proposal
    leaves A^-1 and the tracked value alone)."""
    from paper_2602_05255_amd import inputs as gen
    g = gen.generator(3100 + (kind == "pf"))
    n, L, W = 10, 24, 9
    if kind == "det":
        table = gen.normal(g, (L, n), True)
        occ, emp = gen.occupancy(g, W, L, n)
        chain = oracle.DetChain(table, occ, emp)
    else:
        table = gen.skew_from(gen.normal(g, (L, L), True))
        occ, emp = gen.occupancy(g, W, L, n)
        chain = oracle.PfChain(table, occ, emp)
    for t in range(6):
        k, elec, slot = gen.hop_draws(g, W, n, L - n, (1,) if kind == "pf" else (1, 2), 1 if kind == "pf" else 2)
        mask = g.random(W) < 0.5
        mask[t % W] = True
        mask[(t + 1) % W] = False
        inv0, la0, ph0 = chain.inv.copy(), chain.logabs.copy(), chain.phase.copy()
        occ0 = chain.book.occ.copy()
        chain.propose(k, elec, slot)
        chain.accept(k, elec, slot, mask)
        for w in range(W):
            if not mask[w]:
                assert np.array_equal(chain.inv[w], inv0[w]) and chain.logabs[w] == la0[w]
                assert chain.phase[w] == ph0[w] and np.array_equal(chain.book.occ[w], occ0[w])
                continue
            o = chain.book.occ[w]
            a = table[o] if kind == "det" else table[np.ix_(o, o)]
            resid = np.abs(a @ chain.inv[w] - np.eye(n)).max()
            assert resid <= 1e-10 * np.linalg.cond(a), (t, w, resid)
            sg, lg = np.linalg.slogdet(a)
            want = lg if kind == "det" else 0.5 * lg
            assert abs(chain.logabs[w] - want) <= 1e-10 * max(1.0, abs(want)), (t, w)
            if kind == "pf":
                assert np.array_equal(chain.inv[w], -chain.inv[w].T)
                assert abs(chain.phase[w] ** 2 - sg) <= 1e-10     # pf^2 = det (App. A)
            else:
                assert abs(chain.phase[w] - sg) <= 1e-10
