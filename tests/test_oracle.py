"""Pins for the CPU FP64 oracle: closed forms, brute force, invariants and the
paper's printed values. Nothing here touches the GPU or the HIP library."""

import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

TINY = [
    ((5,), 1), ((8,), 2), ((3, 4), 1), ((4, 4), 3), ((5, 3), 2), ((7, 2), 1),
    ((3, 4, 5), 1), ((4, 4, 4), 3), ((2, 3, 2, 3), 1), ((2, 2, 3, 2), 2),
]


def _rand_problem(n, b, nrhs=2, seed=0):
    return wl.iid_coeffs(seed, n, b), wl.vectors(seed + 1, n, b, nrhs)


# ---------------------------------------------------------------------------
# dense operator: special cases with closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,b", [((6,), 1), ((3, 4), 3), ((3, 2, 4), 2)])
def test_dense_delta_is_identity(n, b):
    x = wl.vectors(3, n, b, 2)
    y = oracle.dense_matvec(wl.delta_coeffs(n, b), x)
    np.testing.assert_allclose(y, x, rtol=0, atol=0)


@pytest.mark.parametrize("n,b,r0,a,c", [
    ((6,), 1, (2,), 0, 0), ((6,), 1, (-3,), 0, 0),
    ((4, 5), 3, (1, -2), 0, 2), ((4, 5), 3, (-3, 4), 2, 1),
    ((3, 4, 2), 2, (2, -1, 1), 1, 0),
])
def test_dense_shifted_delta_is_shift(n, b, r0, a, c):
    """t(r0)[a, c] = 1 alone: y[a, i] = x[c, i - r0], zero where i - r0 leaves the grid."""
    x = wl.vectors(4, n, b, 1)
    y = oracle.dense_matvec(wl.shifted_delta_coeffs(n, b, r0, a, c), x)
    want = np.zeros_like(x)
    for i in np.ndindex(*n):
        j = tuple(ii - rr for ii, rr in zip(i, r0))
        if all(0 <= jj < nn for jj, nn in zip(j, n)):
            want[(0, a) + i] = x[(0, c) + j]
    np.testing.assert_array_equal(y, want)


def test_dense_constant_kernel_sums():
    n = (3, 4, 2)
    x = wl.vectors(5, n, 1, 2)
    y = oracle.dense_matvec(wl.constant_coeffs(n, 0.5 - 2j), x)
    want = (0.5 - 2j) * x.sum(axis=(2, 3, 4), keepdims=True) * np.ones_like(x)
    np.testing.assert_allclose(y, want, rtol=1e-13)


@pytest.mark.parametrize("n", [(5,), (3, 4), (4, 2, 3)])
def test_dense_separable_is_kronecker(n):
    """t(r) = prod_l a_l(r_l) gives T = kron over levels of 1-D Toeplitz matrices."""
    f = wl.separable_factors(6, n)
    T = oracle.dense_operator(wl.separable_coeffs(f))
    K = np.ones((1, 1))
    for a, nl in zip(f, n):
        col = a[nl - 1:]          # a(0), a(1), ..., a(n-1): first column
        row = a[nl - 1::-1]       # a(0), a(-1), ..., a(-(n-1)): first row
        K = np.kron(K, scipy.linalg.toeplitz(col, row))
    np.testing.assert_allclose(T, K, rtol=1e-14, atol=1e-14)


def _adjoint_coeffs(t):
    """t^H(r) = t(-r)^H."""
    flipped = t[(slice(None), slice(None)) + (slice(None, None, -1),) * (t.ndim - 2)]
    return np.conj(np.swapaxes(flipped, 0, 1))


@pytest.mark.parametrize("n,b", [((4, 3), 2), ((3, 3, 2), 3)])
def test_dense_adjoint_identity(n, b):
    t, v = _rand_problem(n, b, 1, seed=11)
    u = wl.vectors(13, n, b, 1)
    Tv = oracle.dense_matvec(t, v)
    THu = oracle.dense_matvec(_adjoint_coeffs(t), u)
    lhs = np.vdot(u.ravel(), Tv.ravel())
    rhs = np.vdot(THu.ravel(), v.ravel())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # and the matrix is literally the conjugate transpose
    np.testing.assert_allclose(oracle.dense_operator(_adjoint_coeffs(t)),
                               oracle.dense_operator(t).conj().T, rtol=0, atol=0)


# ---------------------------------------------------------------------------
# embedding and Algorithm 1 against brute force
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,b", TINY)
def test_embed_matches_dense(n, b):
    t, x = _rand_problem(n, b)
    want = oracle.dense_matvec(t, x)
    got = oracle.embed_matvec(t, x)
    assert wl.relative_l2(got, want) < 1e-13


@pytest.mark.parametrize("n,b", TINY)
def test_split_branch_sum_matches_dense(n, b):
    t, x = _rand_problem(n, b, seed=20)
    want = oracle.dense_matvec(t, x)
    got = oracle.split_branch_sum(t, x)
    assert wl.relative_l2(got, want) < 1e-13


@pytest.mark.parametrize("n,b", [((4, 5, 3), 3), ((6, 2), 1)])
def test_embed_with_precomputed_symbol(n, b):
    t, x = _rand_problem(n, b, seed=21)
    np.testing.assert_array_equal(oracle.embed_matvec_with_symbol(oracle.embed_symbol(t), x),
                                  oracle.embed_matvec(t, x))


@pytest.mark.parametrize("n,b", [((5,), 1), ((4, 3), 3), ((3, 4, 2), 2)])
def test_adjoint_generator_is_conjugate_transpose(n, b):
    """t^H(r) = t(-r)^H generates the conjugate transpose of the dense matrix,
    so <u, T v> = <T^H u, v> for any u, v."""
    t = wl.iid_coeffs(22, n, b)
    T = oracle.dense_operator(t)
    TH = oracle.dense_operator(oracle.adjoint_coeffs(t))
    np.testing.assert_array_equal(TH, T.conj().T)
    u, v = wl.vectors(23, n, b, 1), wl.vectors(24, n, b, 1)
    lhs = np.vdot(u, oracle.dense_matvec(t, v))
    rhs = np.vdot(oracle.dense_matvec(oracle.adjoint_coeffs(t), u), v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("n,b", [((1, 5, 4), 3), ((4, 1, 3), 1), ((6, 1), 2)])
def test_size_one_level_reduces_to_fewer_levels(n, b):
    """A level of size 1 has the single offset 0, so the operator is the
    block-Toeplitz operator of the remaining levels with that coefficient
    slice (same memory layout); all three oracle paths agree with it."""
    c = wl.iid_coeffs(71, n, b)
    x = wl.vectors(72, n, b, 2)
    keep = tuple(v for v in n if v > 1)
    c2 = c.reshape((b, b) + tuple(2 * v - 1 for v in keep))
    x2 = x.reshape((2, b) + keep)
    want = oracle.dense_matvec(c2, x2).reshape(x.shape)
    for got in (oracle.dense_matvec(c, x), oracle.embed_matvec(c, x), oracle.split_branch_sum(c, x)):
        assert wl.relative_l2(got, want) < 1e-13


def test_plain_16_config_three_ways():
    """The 16^3 scalar problem: dense, embedding and the branch sum agree."""
    t, x = wl.plain_16()
    want = oracle.dense_matvec(t, x)
    assert wl.relative_l2(oracle.embed_matvec(t, x), want) < 1e-13
    assert wl.relative_l2(oracle.split_branch_sum(t, x), want) < 1e-13


@pytest.mark.parametrize("n", [(6, 5), (4, 3, 5)])
def test_sampled_rows_match_dense(n):
    t, x = _rand_problem(n, 3, seed=30)
    want = oracle.dense_matvec(t, x)
    rng = np.random.default_rng(0)
    pts = np.stack([rng.integers(0, v, 7) for v in n], axis=1)
    got = oracle.sampled_rows(t, x, pts)
    ref = np.stack([want[(slice(None), slice(None)) + tuple(p)] for p in pts], axis=-1)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_green_kernel_gives_complex_symmetric_matrix():
    """Green blocks are symmetric and even in r: u^T (T v) = (T u)^T v."""
    n = (5, 4, 3)
    t = wl.green_coeffs(n, 0.7)
    u = wl.vectors(40, n, 3, 1)
    v = wl.vectors(41, n, 3, 1)
    lhs = np.sum(u * oracle.embed_matvec(t, v))
    rhs = np.sum(oracle.embed_matvec(t, u) * v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_skew_kernel_gives_complex_symmetric_matrix():
    """[rhat]_x blocks: t(r)^T = -t(r) and t(-r) = -t(r), so T^T = T as well."""
    n = (4, 5, 3)
    t = wl.skew_coeffs(n, 1.3)
    u = wl.vectors(42, n, 3, 1)
    v = wl.vectors(43, n, 3, 1)
    lhs = np.sum(u * oracle.dense_matvec(t, v))
    rhs = np.sum(oracle.dense_matvec(t, u) * v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ---------------------------------------------------------------------------
# Section II.A identities
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nl", [1, 2, 3, 7, 16, 40])
def test_split_property(nl):
    """Even bins of the 2n-point DFT of [v, 0] are F(v); odd bins are F(P v)."""
    v = wl.complex_normal(np.random.default_rng(nl), (nl,))
    F = np.fft.fft(np.concatenate([v, np.zeros(nl)]))
    np.testing.assert_allclose(F[0::2], np.fft.fft(v), atol=1e-12)
    np.testing.assert_allclose(F[1::2], np.fft.fft(oracle.phase(nl) * v), atol=1e-12)
    # the opposite sign of the phase does not give the odd bins
    if nl > 1:
        assert np.abs(F[1::2] - np.fft.fft(np.conj(oracle.phase(nl)) * v)).max() > 1e-3


@pytest.mark.parametrize("nl", [1, 4, 5, 32])
def test_merge_property(nl):
    """First n entries of the 2n-point inverse DFT of Y = (Y_e + conj(P) Y_o) / 2
    computed with n-point inverses of the even and odd bins."""
    Y = wl.complex_normal(np.random.default_rng(100 + nl), (2 * nl,))
    y = np.fft.ifft(Y)[:nl]
    ym = 0.5 * (np.fft.ifft(Y[0::2]) + np.conj(oracle.phase(nl)) * np.fft.ifft(Y[1::2]))
    np.testing.assert_allclose(ym, y, atol=1e-14)


def test_embedded_generator_places_offsets_mod_2n():
    n = (3,)
    t = np.arange(1, 6).reshape(1, 1, 5).astype(np.complex128)  # r = -2..2 -> 1..5
    c = oracle.embedded_generator(t)[0, 0]
    # positions: r=0 ->0, 1 ->1, 2 ->2, pad 3, r=-2 ->4, r=-1 ->5
    np.testing.assert_array_equal(c, [3, 4, 5, 0, 1, 2])


def test_two_level_symmetry_example():
    """The embedded generator of an even 2-level generator has the mirror
    pattern of the paper's two-level example (golden fixture)."""
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "two_level_symmetry.txt"))
            if ln.strip() and not ln.startswith("#")]
    n = (4, 4)
    # f^{ij} encoded as the distinct value 10*i + j + 1 for |r_1| = i, |r_2| = j
    r1, r2 = wl.offsets(n)
    t = (10 * np.abs(r1) + np.abs(r2) + 1).astype(np.complex128)[None, None]
    c = oracle.embedded_generator(t)[0, 0].real.astype(int)
    for m1 in range(8):
        for m2 in range(8):
            lab = rows[m1][m2]
            want = 0 if lab == "0" else 10 * int(lab[0]) + int(lab[1]) + 1
            assert c[m1, m2] == want, (m1, m2)


# ---------------------------------------------------------------------------
# Section II.C: counts, memory, ratios
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,nl", [(1, 8), (2, 4), (3, 4), (4, 2), (3, 8), (6, 2)])
def test_lazy_order_counts_match_c_split(d, nl):
    """The lazy evaluation's work equals Eq. (CompRatio)'s C_split exactly,
    with 2^l forward and 2^l inverse FFTs at level l, 2^(d+1) - 2 phase
    passes (a split and a merge per inner node) and at most d + 1 live
    vectors (Section II.C)."""
    n = (nl,) * d
    cnt = oracle.lazy_costs(n)
    s = nl ** d
    assert cnt["total"] == pytest.approx(oracle.c_split(n), rel=1e-15)
    assert cnt["total"] == pytest.approx(oracle.c_split_closed(nl, d), rel=1e-15)
    assert cnt["mult"] == 2 ** d * s
    assert cnt["phase"] == 2 * (2 ** d - 1) * s
    for level in range(1, d + 1):
        assert cnt["fft_calls"][level] == 2 ** level
        assert cnt["ifft_calls"][level] == 2 ** level
    assert cnt["peak"] == d + 1
    assert cnt["live_at_end"] == 1


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_lazy_order_structure(d):
    """Every leaf once, in increasing branch index (even child before odd);
    every level's transforms bracket properly (an inverse only after a forward
    of the same level, never two forwards in a row on one level); a merge at
    level l only after both children at level l were closed."""
    ev = oracle.lazy_order(d)
    assert [q for k, q in ev if k == "leaf"] == list(range(2 ** d))
    open_ = {l: 0 for l in range(1, d + 1)}
    closed_children = {l: 0 for l in range(1, d + 1)}
    for k, a in ev:
        if k == "fft":
            assert open_[a] == 0
            open_[a] = 1
        elif k == "ifft":
            assert open_[a] == 1
            open_[a] = 0
            closed_children[a] += 1
        elif k == "merge":
            assert closed_children[a] == 2
            closed_children[a] = 0
        elif k == "leaf":
            assert all(open_.values())
    assert not any(open_.values())


def test_lazy_costs_scale_with_blocks_and_rhs():
    n = (4, 4, 4)
    cnt = oracle.lazy_costs(n, b=3, nrhs=2)
    base = oracle.c_split(n) - 8 * 64
    assert cnt["fft"] + cnt["phase"] == pytest.approx(3 * 2 * base)
    assert cnt["mult"] == 2 * 9 * 8 * 64
    assert cnt["peak"] == 4


def test_table_one():
    g = json.load(open(os.path.join(GOLDEN, "table1.json")))
    for i, d in enumerate(g["d"]):
        # printed to two decimals (half up: 65/8 = 8.125 is printed 8.13)
        assert abs(oracle.ratio_c_asymptotic(d) - g["R_c"][i]) <= 0.005 + 1e-12
        assert abs(oracle.ratio_m(d) - g["R_m"][i]) <= 0.005 + 1e-12
        assert abs(oracle.ratio_m_sym(d) - g["R_m_sym"][i]) <= 0.005 + 1e-12
    o = g["outlook_d3"]
    assert oracle.ratio_c_asymptotic(3) == pytest.approx(o["R_c"][0] / o["R_c"][1], rel=1e-15)
    assert oracle.ratio_m(3) == pytest.approx(o["R_m"][0] / o["R_m"][1], rel=1e-15)
    assert oracle.ratio_m_sym(3) == pytest.approx(o["R_m_sym"][0] / o["R_m_sym"][1], rel=1e-15)


def test_ratio_c_second_form_and_limit():
    for d in range(1, 7):
        for nl in (4, 64, 1024):
            # the paper's simplified form divides numerator and denominator by 2^(d+1) s
            lg = math.log2(nl)
            simplified = (d * math.log2(2 * nl) + 0.5) / ((1 - 2.0 ** -d) * (2 * lg + 1) + 0.5)
            assert oracle.ratio_c(nl, d) == pytest.approx(simplified, rel=1e-13)
        assert oracle.ratio_c(2 ** 40, d) == pytest.approx(oracle.ratio_c_asymptotic(d), rel=0.03)
    assert oracle.ratio_c(64, 3) == pytest.approx(1.811, abs=5e-4)


def test_memory_models_reproduce_ratios():
    for d in range(2, 7):
        n = (8,) * d
        e, s = oracle.mem_embed(n), oracle.mem_split(n)
        assert (e["vectors"] + e["symbol"]) / (s["vectors"] + s["symbol"]) == \
            pytest.approx(oracle.ratio_m(d))
        s1 = 8 ** d
        assert (e["vectors"] + s1) / (s["vectors"] + s1) == pytest.approx(oracle.ratio_m_sym(d))


# ---------------------------------------------------------------------------
# symmetric / skew-symmetric storage
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [(4, 6), (5, 4, 3), (4, 4, 4)])
def test_green_symbol_compression_roundtrip(n):
    t = wl.green_coeffs(n, 0.7)
    par = wl.green_parity(len(n)) if len(n) == 3 else wl.green_parity(2)
    C = oracle.embed_symbol(t)
    comp = oracle.compress_symbol(C, par)
    np.testing.assert_allclose(oracle.expand_symbol(comp, par, n), C, atol=1e-12)
    stored = sum(v.size for v in comp.values())
    assert stored == 9 * math.prod(v + 1 for v in n)


@pytest.mark.parametrize("n", [(4, 5, 3), (6, 6, 4)])
def test_skew_symbol_compression_roundtrip(n):
    t = wl.skew_coeffs(n, 1.3)
    par = wl.skew_parity(3)
    C = oracle.embed_symbol(t)
    comp = oracle.compress_symbol(C, par)
    np.testing.assert_allclose(oracle.expand_symbol(comp, par, n), C, atol=1e-12)


def test_odd_generator_with_nonzero_centre_plane():
    """Odd along level 1 apart from its r_1 = 0 plane: C^[2n - m] = 2 C^[0] - C^[m]."""
    n = (5, 4)
    rng = np.random.default_rng(7)
    r1, r2 = wl.offsets(n)
    g = wl.complex_normal(rng, (n[0], 2 * n[1] - 1))  # g(|r_1|, r_2)
    f = wl.complex_normal(rng, (2 * n[1] - 1,))
    t = np.sign(r1) * g[np.abs(r1[:, 0])][:, :] + (r1 == 0) * f[None, :]
    t = t[None, None].astype(np.complex128)
    par = np.array([[[2, 0]]])
    C = oracle.embed_symbol(t)
    comp = oracle.compress_symbol(C, par)
    np.testing.assert_allclose(oracle.expand_symbol(comp, par, n), C, atol=1e-12)
    # the naive sign flip is wrong when the centre plane is not zero
    naive = oracle.expand_symbol(comp, np.array([[[2, 0]]]), n)
    flip = naive.copy()
    flip[0, 0, n[0] + 1:] = -C[0, 0, 1:n[0]][::-1]
    assert np.abs(flip - C).max() > 1e-3


def test_branch_symbols_are_parity_sublattices():
    n = (3, 4)
    t = wl.iid_coeffs(60, n, 2)
    C = oracle.embed_symbol(t)
    Tb = oracle.branch_symbols(t)
    assert Tb.shape == (4, 2, 2, 3, 4)
    np.testing.assert_array_equal(Tb[oracle.branch_index((1, 0))], C[:, :, 1::2, 0::2])
    np.testing.assert_array_equal(Tb[oracle.branch_index((0, 1))], C[:, :, 0::2, 1::2])


# ---------------------------------------------------------------------------
# the pins catch plausible mistakes (mutations planted in the oracle, on the CPU)
# ---------------------------------------------------------------------------

def test_pins_catch_wrong_phase_sign(monkeypatch):
    t, x = _rand_problem((4, 5), 1, 1, seed=70)
    want = oracle.dense_matvec(t, x)
    from oracle import toeplitz as tp
    monkeypatch.setattr(tp, "phase", lambda nl: np.exp(1j * np.pi * np.arange(nl) / nl))
    assert wl.relative_l2(tp.split_branch_sum(t, x), want) > 1e-2


def test_pins_catch_transposed_blocks():
    t, x = _rand_problem((3, 4), 3, 1, seed=71)
    want = oracle.dense_matvec(t, x)
    bad = np.swapaxes(t, 0, 1).copy()
    assert wl.relative_l2(oracle.embed_matvec(bad, x), want) > 1e-2
    assert wl.relative_l2(oracle.split_branch_sum(bad, x), want) > 1e-2


@pytest.mark.parametrize("kind,n", [("green", (4, 5, 3)), ("green", (5, 4)), ("skew", (4, 3, 5))])
def test_declared_parity_masks_hold(kind, n):
    """workloads' parity masks: flipping offset axis l maps t to +t (even) or -t (odd)."""
    d = len(n)
    if kind == "green":
        t, par = wl.green_coeffs(n, 0.7), wl.green_parity(d)
    else:
        t, par = wl.skew_coeffs(n, 1.3), wl.skew_parity(d)
    for a in range(3):
        for c in range(3):
            for l in range(d):
                flipped = np.flip(t[a, c], axis=l)
                sign = 1.0 if par[a, c, l] == wl.EVEN else -1.0
                # exactly: plan creation verifies a declared mask bit for bit
                np.testing.assert_array_equal(flipped, sign * t[a, c])


def test_stored_large_rows_match_direct_sums():
    """tests/golden/large_256_rows.npz (written by make_large_rows.py from the
    embedding oracle) agrees with direct sums over the whole 256 x 256 x 128
    grid at two of its points (a corner and an interior point) for the first
    and last right-hand side of both kernels."""
    g = np.load(os.path.join(GOLDEN, "large_256_rows.npz"), allow_pickle=False)
    cfg = wl.LARGE_256
    n = cfg["n"]
    assert tuple(g["n"]) == n and g["points"].shape == (128, 3)
    pts = g["points"]
    pick = [0, 100]
    assert tuple(pts[0]) == (0, 0, 0)
    x = wl.vectors(cfg["seed_x"], n, 3, cfg["nrhs"])[[0, cfg["nrhs"] - 1]]
    for name, make in (("green", wl.green_coeffs), ("skew", wl.skew_coeffs)):
        coeffs = make(n, cfg["k"])
        rows = oracle.sampled_rows(coeffs, x, pts[pick])
        want = g[name][[0, cfg["nrhs"] - 1]][:, :, pick]
        assert wl.relative_l2(rows, want) < 1e-12
        del coeffs
