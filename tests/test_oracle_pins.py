"""Pins of the FP64 oracle against facts fixed by the paper and by the
mathematics, independent of the oracle's own code paths.

Each test names the passage it pins. A plausible slip in the oracle (wrong
sign in the twiddles, a transposed operand, a dropped weight, a wrong
denominator, a wrong update sign, an off-centre window) fails at least one.
"""
import cmath
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import cfse, spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed=0):
    return np.random.default_rng(seed)


def _brute_dft(x, F):
    """Double sum over the area of x[m,n]*exp(-j2pi(km+ln)/F), plain loops."""
    M, N = x.shape
    X = np.zeros((F, F), dtype=complex)
    for k in range(F):
        for l in range(F):
            acc = 0j
            for m in range(M):
                for n in range(N):
                    acc += complex(x[m, n]) * cmath.exp(-2j * math.pi * (k * m + l * n) / F)
            X[k, l] = acc
    return X


# --------------------------------------------------------------- eq. (7)

@pytest.mark.parametrize("F,M,N", [(4, 3, 2), (4, 4, 4), (8, 5, 7), (8, 8, 8)])
def test_projection_is_dft_bruteforce(F, M, N):
    """eq. (7): the projection onto phi* is the unnormalised DFT; the
    separable oracle projection equals the brute-force double sum and
    numpy's FFT of the zero-padded area."""
    rng = _rng(F * 100 + M * 10 + N)
    x = rng.normal(size=(M, N)) + 1j * rng.normal(size=(M, N))
    got = cfse.project(x, cfse.analysis_matrix(F, M), cfse.analysis_matrix(F, N))
    brute = _brute_dft(x, F)
    pad = np.zeros((F, F), dtype=complex)
    pad[:M, :N] = x
    np.testing.assert_allclose(got, brute, atol=1e-12)
    np.testing.assert_allclose(got, np.fft.fft2(pad), atol=1e-12)


def test_parseval():
    """Energy of the area equals the spectrum energy divided by F^2."""
    rng = _rng(3)
    F, M, N = 16, 11, 13
    x = rng.normal(size=(M, N))
    X = cfse.project(x, cfse.analysis_matrix(F, M), cfse.analysis_matrix(F, N))
    assert abs(np.sum(np.abs(x) ** 2) - np.sum(np.abs(X) ** 2) / F ** 2) < 1e-10 * np.sum(x ** 2)


def test_basis_products():
    """eqs. (5), (6): phi_a phi_b = phi_(a+b), phi_a phi_b* = phi_(a-b), mod F."""
    F, M, N = 8, 5, 6
    a, b = (3, 5), (6, 7)
    pa = cfse.basis(F, M, N, *a)
    pb = cfse.basis(F, M, N, *b)
    np.testing.assert_allclose(pa * pb, cfse.basis(F, M, N, (a[0] + b[0]) % F, (a[1] + b[1]) % F), atol=1e-14)
    np.testing.assert_allclose(pa * np.conj(pb), cfse.basis(F, M, N, (a[0] - b[0]) % F, (a[1] - b[1]) % F), atol=1e-14)
    # eq. (1): explicit exponential
    m, n = 4, 5
    assert abs(pa[m, n] - cmath.exp(2j * math.pi * (a[0] * m + a[1] * n) / F)) < 1e-14


def test_orthogonality_full_grid():
    """eq. (16): on the full F x F grid distinct basis functions are
    orthogonal and each has energy F*F."""
    F = 8
    for (u, v), (k, l) in [((1, 2), (1, 2)), ((1, 2), (3, 2)), ((0, 0), (7, 7))]:
        s = np.sum(cfse.basis(F, F, F, u, v) * np.conj(cfse.basis(F, F, F, k, l)))
        assert abs(s - (F * F if (u, v) == (k, l) else 0)) < 1e-12


# --------------------------------------------------------------- eq. (3)

def test_window_closed_form():
    """eq. (3): the four centre pixels of an even-sized area sit sqrt(0.5)
    from the centre, the corner sqrt(2)*(M-1)/2; odd sizes have weight 1
    at the centre."""
    rho = 0.8
    w = cfse.window(48, 48, rho)
    for m, n in [(23, 23), (23, 24), (24, 23), (24, 24)]:
        assert w[m, n] == pytest.approx(rho ** math.sqrt(0.5), rel=1e-15)
    assert w[0, 0] == pytest.approx(rho ** (math.sqrt(2) * 23.5), rel=1e-14)
    assert w[47, 0] == pytest.approx(w[0, 0], rel=1e-15)
    w2 = cfse.window(5, 7, rho)
    assert w2[2, 3] == 1.0
    assert w2[0, 3] == pytest.approx(rho ** 2, rel=1e-15)
    assert w2[2, 0] == pytest.approx(rho ** 3, rel=1e-15)


def test_weighting_masks_loss_and_frame_edge():
    """eq. (3) and the block geometry: w = 0 on B, on lost pixels of other
    blocks and outside the frame."""
    frames = np.full((1, 40, 40), 100, dtype=np.uint8)
    avail = np.ones_like(frames)
    avail[0, 10:12, 28:30] = 0      # pixels of another lost block inside the area
    blk = dict(frame=0, y0=4, x0=32, bh=4, bw=4, border=6, fft=32, iters=1)
    s, A, B = cfse.area_of_block(frames, avail, blk)   # area rows -2..13, cols 26..41
    assert s.shape == (16, 16)
    assert B.sum() == 16 and not (A & B).any()
    assert not A[:, 14:].any()                # x >= 40 lies outside the frame
    assert not A[0:2, :].any()                # y < 0 lies outside the frame
    assert not A[12:14, 2:4].any()            # the other block's lost pixels
    assert A.sum() == 16 * 16 - 16 - 2 * 16 - 2 * 14 + 0 - 4
    w = cfse.weighting(16, 16, 0.8, A)
    assert (w[~A] == 0).all() and (w[A] > 0).all()


# --------------------------------------------------------------- iteration algebra

def _patch(seed=0, M=12, N=12, hole=4, F=16):
    rng = _rng(seed)
    y, x = np.mgrid[0:M, 0:N]
    s = 100 + 30 * np.sin(2 * np.pi * x / 7.3 + 1) + 20 * np.cos(2 * np.pi * y / 5.1) + rng.normal(0, 2, (M, N))
    A = np.ones((M, N), dtype=bool)
    b0 = (M - hole) // 2
    A[b0:b0 + hole, b0:b0 + hole] = False
    w = cfse.weighting(M, N, 0.8, A)
    return s, w, F


@pytest.mark.parametrize("gamma", [0.2, 0.5, 1.0])
def test_energy_identity_and_monotone(gamma):
    """Weighted least squares along one basis function (eqs. (9), (13),
    (17)) lowers the weighted residual energy sum(w|r|^2) by exactly
    gamma*(2-gamma)*|R_w[u,v]|^2/W0 with W0 = sum(w) and R_w[u,v] =
    W0*c/gamma; hence it never increases for 0 < gamma <= 1."""
    s, w, F = _patch()
    res = cfse.cfse(s, w, F, gamma, 60)
    W0 = w.sum()
    E = np.array(res["energy"])
    for nu, c in enumerate(res["chat"]):
        R = W0 * c / gamma
        expect = E[nu] - gamma * (2 - gamma) * abs(R) ** 2 / W0
        assert abs(E[nu + 1] - expect) <= 1e-10 * E[0]
    assert np.all(np.diff(E) <= 1e-12 * E[0])


def test_selection_is_bruteforce_least_squares():
    """eq. (10): the selected basis function gives the largest drop of the
    weighted residual energy when fitted alone by weighted least squares;
    eq. (13): the coefficient is gamma times that fit. Checked with an
    independent dense least-squares solve per candidate."""
    s, w, F = _patch(seed=5, M=6, N=6, hole=2, F=8)
    gamma = 0.7
    res = cfse.cfse(s, w, F, gamma, 6)
    M, N = s.shape
    sw = np.sqrt(w).ravel()
    r = s.astype(complex)
    for nu in range(6):
        drops = np.zeros(F * F)
        fits = np.zeros(F * F, dtype=complex)
        for idx in range(F * F):
            k, l = divmod(idx, F)
            phi = np.array([[cmath.exp(2j * math.pi * (k * m + l * n) / F) for n in range(N)] for m in range(M)])
            A = (sw * phi.ravel())[:, None]
            b = sw * r.ravel()
            c, *_ = np.linalg.lstsq(A, b, rcond=None)
            fits[idx] = c[0]
            drops[idx] = np.sum(np.abs(b) ** 2) - np.sum(np.abs(b - A[:, 0] * c[0]) ** 2)
        best = np.flatnonzero(drops >= drops.max() * (1 - 1e-9))
        assert res["seq"][nu] == best[0]
        assert abs(res["chat"][nu] - gamma * fits[best[0]]) < 1e-9 * abs(fits[best[0]])
        k, l = divmod(best[0], F)
        phi = np.array([[cmath.exp(2j * math.pi * (k * m + l * n) / F) for n in range(N)] for m in range(M)])
        r = r - gamma * fits[best[0]] * phi


def test_worked_example_f2_golden():
    """Hand-derived 2x2 example (tests/golden/f2_worked_example.txt)."""
    rows, G, E = [], None, None
    with open(os.path.join(GOLDEN, "f2_worked_example.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            if f[0] == "G":
                G = Fraction(int(f[1]), int(f[2]))
            elif f[0] == "E":
                E = (Fraction(int(f[1]), int(f[2])), Fraction(int(f[3]), int(f[4])))
            else:
                rows.append((int(f[1]), int(f[2]), Fraction(int(f[3]), int(f[4]))))
    for rho in (0.8, 0.3, 1.0):
        s = np.array([[4.0, 2.0], [1.0, 77.0]])      # s(1,1) is lost: any value
        A = np.array([[True, True], [True, False]])
        w = cfse.weighting(2, 2, rho, A)
        omega = rho ** math.sqrt(0.5)
        res = cfse.cfse(s, w, 2, 0.5, 3)
        for (k, l, c), idx, got in zip(rows, res["seq"], res["chat"]):
            assert idx == k * 2 + l
            assert abs(got - float(c)) < 1e-13
        assert abs(res["g"][1, 1] - float(G)) < 1e-13
        assert abs(res["energy"][0] - float(E[0]) * omega) < 1e-12
        assert abs(res["energy"][1] - float(E[1]) * omega) < 1e-12


# --------------------------------------------------------------- special cases

@pytest.mark.parametrize("k0,l0", [(3, 5), (0, 0), (8, 1)])
def test_single_basis_function(k0, l0):
    """A complex input equal to a*phi_(k0,l0) on the area: every iteration
    selects (k0,l0) (the shifted window spectrum is smaller than W0 off DC),
    the accumulated coefficient after nu iterations is a*(1-(1-gamma)^nu),
    and gamma = 1 recovers the signal exactly in one iteration, B included."""
    F, M, N = 16, 12, 12
    a = 37.5 - 12.25j
    A = np.ones((M, N), dtype=bool)
    A[4:8, 4:8] = False
    w = cfse.weighting(M, N, 0.8, A)
    s = a * cfse.basis(F, M, N, k0, l0)
    for gamma in (0.3, 0.5):
        res = cfse.cfse(s, w, F, gamma, 10)
        assert all(i == k0 * F + l0 for i in res["seq"])
        acc = np.cumsum(res["chat"])
        for nu in range(10):
            assert abs(acc[nu] - a * (1 - (1 - gamma) ** (nu + 1))) < 1e-12 * abs(a)
    res = cfse.cfse(s, w, F, 1.0, 1)
    np.testing.assert_allclose(res["g"], s, atol=1e-12 * abs(a))


def test_real_cosine_picks_lower_conjugate():
    """A real cosine has two conjugate projections of equal size; the tie
    goes to the lower linear index, and the second pick is its partner."""
    F, M, N = 16, 12, 12
    A = np.ones((M, N), dtype=bool)
    A[4:8, 4:8] = False
    w = cfse.weighting(M, N, 0.8, A)
    k0, l0 = 13, 2                       # partner (3, 14) has the lower index
    s = 50.0 * cfse.basis(F, M, N, k0, l0).real
    res = cfse.cfse(s, w, F, 0.5, 2)
    lo = min(k0 * F + l0, ((-k0) % F) * F + (-l0) % F)
    hi = max(k0 * F + l0, ((-k0) % F) * F + (-l0) % F)
    assert res["seq"][0] == lo
    assert res["gap"][0] < 1e-12


def test_placement_covariance():
    """Moving the area by (a, b) inside the transform grid multiplies every
    projection by the unit phase exp(-j2pi(ka+lb)/F): same selections, same
    model on the area, coefficients rotated by that phase."""
    s, w, F = _patch(seed=2)
    base = cfse.cfse(s, w, F, 0.5, 25)
    a, b = 3, 2
    moved = cfse.cfse(s, w, F, 0.5, 25, offset=(a, b))
    assert moved["seq"] == base["seq"]
    for idx, c0, c1 in zip(base["seq"], base["chat"], moved["chat"]):
        u, v = divmod(idx, F)
        assert abs(c1 - c0 * cmath.exp(-2j * math.pi * (u * a + v * b) / F)) < 1e-10 * abs(c0)
    np.testing.assert_allclose(moved["g"], base["g"], atol=1e-9)


def test_homogeneity():
    """Scaling the signal scales every coefficient and keeps the selections."""
    s, w, F = _patch(seed=4)
    base = cfse.cfse(s, w, F, 0.5, 20)
    scaled = cfse.cfse(-2.5 * s, w, F, 0.5, 20)
    assert scaled["seq"] == base["seq"]
    np.testing.assert_allclose(scaled["chat"], -2.5 * np.array(base["chat"]), rtol=1e-11)


def test_degenerate_cases():
    """gamma = 0 and I = 0 leave the model at zero; rho = 1 makes w the
    indicator of A; an empty support is an error."""
    s, w, F = _patch(seed=6)
    res = cfse.cfse(s, w, F, 0.0, 5)
    assert np.all(np.array(res["chat"]) == 0) and np.all(res["g"] == 0)
    res = cfse.cfse(s, w, F, 0.5, 0)
    assert res["seq"] == [] and np.all(res["g"] == 0)
    A = w > 0
    assert np.array_equal(cfse.weighting(*A.shape, 1.0, A), A.astype(float))
    with pytest.raises(ValueError):
        cfse.cfse(s, np.zeros_like(w), F, 0.5, 1)


def test_window_spectrum_properties():
    """W = DFT(w) (eq. (11)): W[0,0] = sum(w) is the denominator of eq. (9),
    and W[-k,-l] = conj(W[k,l]) for real w."""
    s, w, F = _patch(seed=7)
    M, N = w.shape
    Wf = cfse.project(w, cfse.analysis_matrix(F, M), cfse.analysis_matrix(F, N))
    assert abs(Wf[0, 0] - w.sum()) < 1e-12 * w.sum()
    idx = (-np.arange(F)) % F
    np.testing.assert_allclose(Wf[np.ix_(idx, idx)], np.conj(Wf), atol=1e-11)


def test_independence_from_outside_area():
    """A block's result depends only on its own area: changing pixels outside
    it, or lost pixels inside it, changes nothing."""
    from synth import workloads
    wl = workloads.isolated_256()
    blk = wl.blocks[27]
    base = cfse.extrapolate_block(wl.frames, wl.avail, blk, 0.8, 0.5, iters=30)
    frames = wl.frames.copy()
    frames[0, :int(blk["y0"]) - 17, :] = 7                 # outside the area
    frames[wl.avail == 0] = 255                             # every lost pixel
    other = cfse.extrapolate_block(frames, wl.avail, blk, 0.8, 0.5, iters=30)
    assert other["seq"] == base["seq"]
    np.testing.assert_array_equal(other["values"], base["values"])


# ------------------------------------------ warm start and restricted bins

def test_init_continues_an_interrupted_run():
    """Initial coefficients (eq. (8) with a non-zero starting model): I1
    iterations, then I2 more started from the first run's accumulated
    coefficients, equal one uninterrupted run of I1 + I2 iterations (the
    residual is s minus the model either way)."""
    s, w, F = _patch(seed=8)
    first = cfse.cfse(s, w, F, 0.5, 15)
    rest = cfse.cfse(s, w, F, 0.5, 20, init=dict(first["coefs"]))
    whole = cfse.cfse(s, w, F, 0.5, 35)
    assert rest["seq"] == whole["seq"][15:]
    np.testing.assert_allclose(rest["chat"], whole["chat"][15:], rtol=1e-10, atol=1e-10 * abs(whole["chat"][0]))
    np.testing.assert_allclose(rest["g"], whole["g"], atol=1e-9)
    assert abs(rest["energy"][0] - whole["energy"][15]) <= 1e-10 * whole["energy"][0]


def test_init_single_basis_function():
    """Starting from c0 on the basis function the signal is made of: with no
    iteration the model is c0*phi; with iterations the remaining amplitude
    a - c0 shrinks by (1 - gamma) per step, so the accumulated coefficient is
    a - (a - c0)(1 - gamma)^nu."""
    F, M, N = 16, 12, 12
    k0, l0, a, c0 = 5, 11, 40.0 + 9.0j, 30.0 - 2.0j
    A = np.ones((M, N), dtype=bool)
    A[4:8, 4:8] = False
    w = cfse.weighting(M, N, 0.8, A)
    phi = np.exp(2j * np.pi * (k0 * np.arange(M)[:, None] + l0 * np.arange(N)[None, :]) / F)
    s = a * phi
    res = cfse.cfse(s, w, F, 0.5, 0, init={(k0, l0): c0})
    np.testing.assert_allclose(res["g"], c0 * phi, atol=1e-12 * abs(c0))
    res = cfse.cfse(s, w, F, 0.5, 6, init={(k0, l0): c0})
    assert res["seq"] == [k0 * F + l0] * 6
    acc = c0 + np.cumsum(res["chat"])
    for nu in range(6):
        assert abs(acc[nu] - (a - (a - c0) * 0.5 ** (nu + 1))) < 1e-12 * abs(a)
    assert abs(res["coefs"][(k0, l0)] - acc[-1]) < 1e-12 * abs(a)


def test_candidate_mask_all_true_is_unrestricted():
    """An all-true candidate mask restricts nothing: identical selections
    and coefficients, bit for bit."""
    s, w, F = _patch(seed=9)
    free = cfse.cfse(s, w, F, 0.5, 30)
    allc = cfse.cfse(s, w, F, 0.5, 30, cand=np.ones((F, F), dtype=bool))
    assert free["seq"] == allc["seq"] and free["chat"] == allc["chat"]


def test_single_candidate_converges_to_its_fixed_point():
    """Input a*phi_0 + b*phi_1 with the stronger b, restricted to the single
    candidate phi_0: every step selects phi_0, and its accumulated
    coefficient is C*(1 - (1 - gamma)^nu) with C* = a + b*Wd/W0, where
    W0 = sum(w) and Wd is the window's DFT at the difference of the two
    bins (brute-force double sum), the weighted least-squares fit of phi_0
    alone."""
    F, M, N = 8, 6, 7
    k0, l0, k1, l1 = 1, 2, 3, 6
    a, b = 10.0 - 4.0j, 25.0 + 15.0j
    A = np.ones((M, N), dtype=bool)
    A[2:4, 3:5] = False
    w = cfse.weighting(M, N, 0.7, A)
    m, n = np.arange(M)[:, None], np.arange(N)[None, :]
    phi = lambda k, l: np.exp(2j * np.pi * (k * m + l * n) / F)
    s = a * phi(k0, l0) + b * phi(k1, l1)
    free = cfse.cfse(s, w, F, 0.5, 1)
    assert free["seq"] == [k1 * F + l1]
    cand = np.zeros((F, F), dtype=bool)
    cand[k0, l0] = True
    Wd = _brute_dft(w, F)[(k0 - k1) % F, (l0 - l1) % F]
    cstar = a + b * Wd / w.sum()
    for gamma in (0.5, 0.9):
        res = cfse.cfse(s, w, F, gamma, 8, cand=cand)
        assert res["seq"] == [k0 * F + l0] * 8
        acc = np.cumsum(res["chat"])
        for nu in range(8):
            assert abs(acc[nu] - cstar * (1 - (1 - gamma) ** (nu + 1))) < 1e-11 * abs(cstar)


def test_candidate_mask_keeps_selections_inside_and_energy_identity():
    """A random candidate mask: every selection lies in it, is the largest
    criterion among the candidates (checked against a brute-force
    projection of the spatial residual), and the weighted residual energy
    falls by gamma(2 - gamma)|R_w[u,v]|^2/W0 per step."""
    s, w, F = _patch(seed=10)
    M, N = s.shape
    rng = _rng(10)
    cand = rng.random((F, F)) < 0.2
    gamma = 0.5
    res = cfse.cfse(s, w, F, gamma, 25, cand=cand)
    W0 = w.sum()
    r = s.astype(complex)
    for nu, (idx, c) in enumerate(zip(res["seq"], res["chat"])):
        assert cand.ravel()[idx]
        R = _brute_dft(r * w, F).ravel()
        mags = np.where(cand.ravel(), np.abs(R), -1.0)
        assert mags[idx] >= mags.max() * (1 - 1e-9)
        assert abs(c - gamma * R[idx] / W0) < 1e-9 * abs(R).max() / W0
        E0, E1 = res["energy"][nu], res["energy"][nu + 1]
        assert abs(E1 - (E0 - gamma * (2 - gamma) * abs(R[idx]) ** 2 / W0)) <= 1e-10 * res["energy"][0]
        u, v = divmod(idx, F)
        r = r - c * np.exp(2j * np.pi * (u * np.arange(M)[:, None] + v * np.arange(N)[None, :]) / F)


def test_shortfall_and_gap_of_a_forced_selection():
    """Near-tie bookkeeping of the replay protocol: on the full F x F grid
    with w = 1 the basis functions are orthogonal and |R_w| at a bin is
    F^2 |amplitude|. With amplitudes 12 and 9 on two bins, forcing the
    weaker one first gives shortfall (|R|max - |R|followed)/|R|max =
    (12 - 9)/12 = 0.25 (not the 0.4375 of squared magnitudes), the free
    choice is the stronger bin, and the top-two gap is also 0.25."""
    F = 8
    w = np.ones((F, F))
    m, n = np.arange(F)[:, None], np.arange(F)[None, :]
    b1, b2 = (2, 3), (5, 1)
    s = 12.0 * np.exp(2j * np.pi * (b1[0] * m + b1[1] * n) / F) \
        + 9.0j * np.exp(2j * np.pi * (b2[0] * m + b2[1] * n) / F)
    i1, i2 = b1[0] * F + b1[1], b2[0] * F + b2[1]
    res = cfse.cfse(s, w, F, 0.5, 2, forced=[i2, i1])
    assert res["free"][0] == i1
    assert abs(res["short"][0] - 0.25) < 1e-12
    assert abs(res["gap"][0] - 0.25) < 1e-12
    # after half of the weaker amplitude is removed: 12 against 4.5, and the
    # followed bin is now the free choice
    assert res["free"][1] == i1 and res["short"][1] == 0.0
    assert abs(res["gap"][1] - 7.5 / 12) < 1e-12


def test_psnr_over_lost_pixels_hand_value():
    """PSNR over the lost pixels, reconstruction clipped to [0, 255] first.
    Lost pixels (avail == 0) with reference 20, 30, 40 and reconstruction
    22, 300 (clipped to 255), 35: errors 2, 225, -5, MSE = 50654/3, PSNR =
    10 log10(255^2 * 3 / 50654) = 5.855879 dB. The received pixel (error
    1000) does not count; a perfect reconstruction gives infinity."""
    from oracle import metrics
    ref = np.array([[10.0, 20.0], [30.0, 40.0]])
    rec = np.array([[1010.0, 22.0], [300.0, 35.0]])
    avail = np.array([[1, 0], [0, 0]], dtype=np.uint8)
    assert abs(metrics.psnr_lost(ref, rec, avail) - 5.8558787) < 1e-6
    assert metrics.psnr_lost(ref, np.where(avail == 0, ref, -5.0), avail) == float("inf")
    # negative values clip to 0: error -20 on one lost pixel only
    rec2 = ref.copy()
    rec2[0, 1] = -7.0
    assert abs(metrics.psnr_lost(ref, rec2, avail) - 10 * math.log10(65025 * 3 / 400)) < 1e-9


# --------------------------------------------------------------- eq. (18)

def test_frequency_domain_update_matches_projection():
    """eq. (18) is eq. (17) followed by eq. (7): after every step, the
    spectral state (residual spectrum updated by the shifted window
    spectrum) equals the projection of the spatial residual s - sum c*phi
    onto every basis function, formed directly from the direct oracle's
    selections and coefficients; the free-running spectral form makes the
    same selections and its model matches (FP64, relative 1e-10)."""
    from synth import workloads
    wl = workloads.isolated_256()
    F = 64
    for bi in (0, 9, 36, 63):
        blk = wl.blocks[bi]
        s, A, B = cfse.area_of_block(wl.frames, wl.avail, blk)
        M, N = s.shape
        w = cfse.weighting(M, N, 0.8, A)
        res = cfse.cfse(s, w, F, 0.5, 100)
        EM, EN = cfse.analysis_matrix(F, M), cfse.analysis_matrix(F, N)
        st = spectral.SpectralState(s, w, F, 0.5)
        r = s.astype(complex)
        scale = np.abs(st.residual).max()
        for nu in range(100):
            if nu % 9 == 0:   # every ninth state against the spatial residual
                direct = cfse.project(r * w, EM, EN)
                assert np.abs(st.residual - direct).max() <= 1e-10 * scale, (bi, nu)
            idx, c = st.advance(res["seq"][nu])
            assert abs(c - res["chat"][nu]) <= 1e-10 * abs(res["chat"][0]), (bi, nu)
            u, v = divmod(res["seq"][nu], F)
            r = r - res["chat"][nu] * cfse.basis(F, M, N, u, v)
        np.testing.assert_allclose(st.model(), res["g"], atol=1e-9)
        bins, coefs, g = spectral.run(s, w, F, 0.5, 100)
        assert bins == res["seq"]
        np.testing.assert_allclose(g, res["g"], atol=1e-9)


# ------------------------------------------------- arbitrary loss shapes

def _strokes_case():
    from synth import workloads
    wl = workloads.strokes_256(iters=30)
    # a tile with both lost and received pixels
    for i, b in enumerate(wl.blocks):
        t = wl.avail[0, b["y0"]:b["y0"] + b["bh"], b["x0"]:b["x0"] + b["bw"]]
        if 0.2 < (t == 0).mean() < 0.8:
            return wl, i
    raise AssertionError("no partially lost tile")


def test_masked_loss_area_reduces_to_the_rectangle():
    """With every pixel of the block's rectangle lost, the mask-driven loss
    area is the rectangle: identical selections and values."""
    from synth import workloads
    wl = workloads.isolated_256(iters=30)
    for i in (5, 27):
        a = cfse.extrapolate_block(wl.frames, wl.avail, wl.blocks[i], 0.8, 0.5)
        b = cfse.extrapolate_block(wl.frames, wl.avail, wl.blocks[i], 0.8, 0.5, masked=True)
        assert a["seq"] == b["seq"]
        np.testing.assert_array_equal(a["values"], b["values"])
        assert b["lost"].all()


def test_masked_loss_area_constant_signal_is_exact():
    """A constant signal with an irregular loss inside the rectangle: the
    first selection is the DC bin and with gamma = 1 its coefficient is the
    constant itself, so every lost pixel is reproduced exactly."""
    wl, i = _strokes_case()
    frames = np.full_like(wl.frames, 123)
    res = cfse.extrapolate_block(frames, wl.avail, wl.blocks[i], 0.8, 1.0, iters=1, masked=True)
    assert res["seq"] == [0]
    lost = res["lost"]
    assert 0 < lost.sum() < lost.size
    np.testing.assert_allclose(res["values"][lost], 123.0, rtol=0, atol=1e-9)


def test_masked_loss_area_uses_received_pixels_of_the_rectangle():
    """Received pixels inside the rectangle are support, not loss: the loss
    mask is exactly the rectangle's lost pixels, the frame output keeps every
    received pixel, and changing a received pixel inside the rectangle
    changes the extrapolation (it is part of eq. (3)'s support)."""
    wl, i = _strokes_case()
    blk = wl.blocks[i]
    y0, x0, bh, bw = (int(blk[k]) for k in ("y0", "x0", "bh", "bw"))
    rect = wl.avail[0, y0:y0 + bh, x0:x0 + bw]
    res = cfse.extrapolate_block(wl.frames, wl.avail, blk, 0.8, 0.5, masked=True)
    assert np.array_equal(res["lost"], rect == 0)
    out = cfse.extrapolate_frames(wl.frames, wl.avail, wl.blocks[i:i + 1], 0.8, 0.5, masked=True)
    recv = wl.avail != 0
    np.testing.assert_array_equal(out[recv], wl.frames[recv].astype(np.float64))
    changed = np.argwhere(rect != 0)[0]
    frames = wl.frames.copy()
    frames[0, y0 + changed[0], x0 + changed[1]] ^= 0x40
    other = cfse.extrapolate_block(frames, wl.avail, blk, 0.8, 0.5, masked=True)
    assert not np.array_equal(other["values"][res["lost"]], res["values"][res["lost"]])


# ------------------------------------------------------------ 3-D (video)

def _vol(**kw):
    from synth import losses
    v = np.zeros(1, dtype=losses.VOLUME_DTYPE)[0]
    for k, x in kw.items():
        v[k] = x
    return v


def test_3d_reduces_to_2d_with_one_frame():
    """A single-frame volume with a one-point temporal transform is the 2-D
    algorithm: the same selections, coefficients and values."""
    from oracle import cfse3
    from synth import workloads
    wl = workloads.isolated_256(iters=25)
    b = wl.blocks[27]
    r2 = cfse.extrapolate_block(wl.frames, wl.avail, b, 0.8, 0.5)
    v = _vol(frame=0, y0=b["y0"], x0=b["x0"], bt=1, bh=b["bh"], bw=b["bw"], border=b["border"],
             tborder=0, fft=b["fft"], fft_t=1, iters=25)
    r3 = cfse3.extrapolate_volume(wl.frames, wl.avail, v, 0.8, 0.5)
    assert r3["seq"] == r2["seq"]
    np.testing.assert_allclose(r3["chat"], r2["chat"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(r3["values"][:, :, 0], r2["values"], rtol=0, atol=1e-9)


def test_3d_projection_is_dft_bruteforce():
    """eq. (7) in 3-D: the separable projection equals the triple sum."""
    from oracle import cfse3
    rng = np.random.default_rng(4)
    M, N, T, F, Ft = 3, 4, 2, 4, 4
    x = rng.normal(size=(M, N, T)) + 1j * rng.normal(size=(M, N, T))
    got = cfse3.project(x, cfse.analysis_matrix(F, M), cfse.analysis_matrix(F, N), cfse.analysis_matrix(Ft, T))
    ref = np.zeros((F, F, Ft), dtype=complex)
    for k in range(F):
        for l in range(F):
            for s in range(Ft):
                for m in range(M):
                    for n in range(N):
                        for t in range(T):
                            ref[k, l, s] += x[m, n, t] * cmath.exp(-2j * math.pi * (k * m / F + l * n / F + s * t / Ft))
    np.testing.assert_allclose(got, ref, atol=1e-12)


@pytest.mark.parametrize("k0,l0,s0", [(0, 0, 0), (3, 5, 1), (7, 1, 3)])
def test_3d_single_basis_function(k0, l0, s0):
    """A signal that is one 3-D basis function on the support is recovered
    exactly in one iteration with gamma = 1, also on the loss volume."""
    from oracle import cfse3
    F, Ft, M, N, T = 8, 4, 6, 6, 4
    phi = cfse3.basis(F, Ft, M, N, T, k0, l0, s0)
    A = np.ones((M, N, T), dtype=bool)
    A[2:4, 2:4, 1:3] = False
    w = np.where(A, cfse3.window(M, N, T, 0.8), 0.0)
    res = cfse3.cfse3(np.where(A, phi, 0), w, F, Ft, 1.0, 1)
    assert res["seq"] == [(k0 * F + l0) * Ft + s0]
    np.testing.assert_allclose(res["g"], phi, atol=1e-12)


def test_3d_energy_monotone():
    """Weighted residual energy never increases for 0 < gamma <= 1."""
    from oracle import cfse3
    rng = np.random.default_rng(9)
    M, N, T = 10, 10, 4
    s = rng.normal(size=(M, N, T)) * 20 + 100
    A = rng.random((M, N, T)) > 0.2
    w = np.where(A, cfse3.window(M, N, T, 0.8), 0.0)
    for gamma in (0.3, 1.0):
        e = cfse3.cfse3(np.where(A, s, 0), w, 16, 8, gamma, 12)["energy"]
        assert all(b <= a * (1 + 1e-12) for a, b in zip(e, e[1:]))


# ------------------------------------------------------------------ rFSE

def _rfse_case(seed=21, M=12, N=10, F=16):
    rng = np.random.default_rng(seed)
    r = rng.normal(size=(M, N)) * 30 + 90
    A = rng.random((M, N)) > 0.25
    A[4:7, 3:6] = False
    w = np.where(A, cfse.window(M, N, 0.8), 0.0)
    return r, w, A, F


def _pair_lstsq(r, w, F, k, l):
    """Brute-force weighted least squares of r on the real span of the pair
    (k, l), (-k, -l): returns (c, energy decrease); the model is
    Re{c phi*} = Re(c) cos(theta) + Im(c) sin(theta)."""
    M, N = r.shape
    m = np.arange(M)[:, None]
    n = np.arange(N)[None, :]
    th = 2 * math.pi * (k * m + l * n) / F
    cols = [np.cos(th).ravel()]
    if not ((2 * k) % F == 0 and (2 * l) % F == 0):
        cols.append(np.sin(th).ravel())
    X = np.stack(cols, axis=1)
    sw = np.sqrt(w.ravel())
    beta = np.linalg.lstsq(X * sw[:, None], r.ravel() * sw, rcond=None)[0]
    res = r.ravel() - X @ beta
    dec = float(np.sum(w.ravel() * r.ravel() ** 2) - np.sum(w.ravel() * res ** 2))
    c = beta[0] + (1j * beta[1] if len(beta) > 1 else 0)
    return c, dec


def test_rfse_pair_fit_is_weighted_least_squares():
    """The closed-form coefficient and energy decrease of every pair equal a
    brute-force weighted least-squares fit on {cos, sin} (one column for the
    four self-conjugate bins); pins the derivation from eq. (2)."""
    from oracle import rfse
    r, w, A, F = _rfse_case()
    M, N = r.shape
    EM, EN = cfse.analysis_matrix(F, M), cfse.analysis_matrix(F, N)
    P = cfse.project(w * r + 0j, EM, EN)
    Q = rfse.double_freq(cfse.project(w + 0j, EM, EN))
    c, dec = rfse.pair_fit(P, float(w.sum()), Q, rfse.self_conjugate(F))
    for k in range(F):
        for l in range(F):
            cb, db = _pair_lstsq(r, w, F, k, l)
            assert abs(c[k, l] - cb) <= 1e-9 * max(1.0, abs(cb)), (k, l, c[k, l], cb)
            assert abs(dec[k, l] - db) <= 1e-9 * max(1.0, abs(db)), (k, l, dec[k, l], db)


@pytest.mark.parametrize("selection", ["power", "decrease"])
def test_rfse_selection_and_energy_identity(selection):
    """Each iteration selects the lower-index bin of the pair with the
    largest brute-force criterion (the weighted residual's |projection|^2
    by eq. (7), or the least-squares decrease), the weighted energy falls by
    exactly gamma (2 - gamma) times the selected pair's decrease, and the
    model stays real."""
    from oracle import rfse
    r, w, A, F = _rfse_case(seed=5)
    s = np.where(A, r, 0.0)
    gamma = 0.6
    res = rfse.rfse(s, w, F, gamma, 6, selection=selection)
    resid = s.copy()
    for it, idx in enumerate(res["seq"]):
        decs = np.array([[_pair_lstsq(resid, w, F, k, l)[1] for l in range(F)] for k in range(F)])
        if selection == "power":
            crit = np.abs(_brute_dft(resid * w, F)) ** 2
        else:
            crit = decs
        assert idx == int(np.flatnonzero(crit.ravel() >= crit.max() * (1 - 1e-9))[0])
        e0, e1 = res["energy"][it], res["energy"][it + 1]
        assert abs((e0 - e1) - gamma * (2 - gamma) * decs.ravel()[idx]) <= 1e-9 * e0
        u, v = divmod(idx, F)
        m = np.arange(s.shape[0])[:, None]
        n = np.arange(s.shape[1])[None, :]
        th = 2 * math.pi * (u * m + v * n) / F
        ch = res["chat"][it]
        resid = resid - (ch.real * np.cos(th) + ch.imag * np.sin(th))
    assert np.isrealobj(res["g"])
    np.testing.assert_allclose(res["g"], s - resid, atol=1e-9)


@pytest.mark.parametrize("selection", ["power", "decrease"])
@pytest.mark.parametrize("k0,l0", [(3, 5), (13, 2), (0, 0), (8, 0), (0, 8), (8, 8)])
def test_rfse_recovers_a_real_sinusoid(k0, l0, selection):
    """A real sinusoid a cos(theta + p) on the support (a constant or an
    alternating pattern for the self-conjugate bins) is the whole model
    after one iteration at gamma = 1, also on the loss area, and the
    selected bin is the lower index of its pair."""
    from oracle import rfse
    M, N, F = 12, 12, 16
    m = np.arange(M)[:, None]
    n = np.arange(N)[None, :]
    th = 2 * math.pi * (k0 * m + l0 * n) / F
    sc = (2 * k0) % F == 0 and (2 * l0) % F == 0
    x = 37.0 * np.cos(th + (0.0 if sc else 0.7)) + (5.0 if (k0, l0) == (0, 0) else 0.0)
    A = np.ones((M, N), dtype=bool)
    A[4:8, 4:8] = False
    w = np.where(A, cfse.window(M, N, 0.8), 0.0)
    res = rfse.rfse(np.where(A, x, 0.0), w, F, 1.0, 1, selection=selection)
    assert res["seq"] == [min(k0 * F + l0, rfse.pair_index(F, k0 * F + l0))]
    np.testing.assert_allclose(res["g"], x, atol=1e-9)


def test_rfse_pairs_tie_exactly():
    """Both bins of a pair have bit-identical decreases (so the tie rule,
    not rounding, picks the lower index)."""
    from oracle import rfse
    r, w, A, F = _rfse_case(seed=8, F=32)
    M, N = r.shape
    EM, EN = cfse.analysis_matrix(F, M), cfse.analysis_matrix(F, N)
    P = cfse.project(w * r + 0j, EM, EN)
    Q = rfse.double_freq(cfse.project(w + 0j, EM, EN))
    _, dec = rfse.pair_fit(P, float(w.sum()), Q, rfse.self_conjugate(F))
    flip = dec[(-np.arange(F)) % F][:, (-np.arange(F)) % F]
    assert np.array_equal(dec, flip)


# ------------------------------------------------------------ fixed point

def _fixed_area(seed=4, M=48, N=48):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, 256, size=(M, N)).astype(np.int64)
    A = rng.random((M, N)) > 0.2
    A[16:32, 16:32] = False
    return s, A


def test_fixed_transform_rounding_and_scale():
    """The two integer passes equal the exact sums (Python integers, same
    integer twiddles) up to the two roundings (|error| <= 0.5 per pass,
    carried through the second pass), and match the FP64 DFT of the same
    input at scale 2^6 within the twiddle quantisation."""
    from oracle import fixed
    s, A = _fixed_area()
    M, N = s.shape
    wq = np.where(A, fixed.window_q(M, N, 0.8), 0)
    zr, zi = s * wq, wq << fixed.IMAG_SHIFT
    Zr, Zi = fixed.transform(zr, zi)
    Tr, Ti = fixed.twiddles_q()
    # exact sums for a few bins, in Python integers
    for k, l in [(0, 0), (1, 0), (0, 5), (7, 33), (63, 62), (32, 32)]:
        ex = 0
        for m in range(M):
            row = 0
            for n in range(N):
                t = complex(int(Tr[(l * n) % 64]), int(Ti[(l * n) % 64]))
                row += complex(int(zr[m, n]), int(zi[m, n])) * t
            ex += row * complex(int(Tr[(k * m) % 64]), int(Ti[(k * m) % 64]))
        ex /= 2.0 ** (fixed.S_ROW + fixed.S_COL)
        bound = 0.5 * math.sqrt(2) * (1 + M * 2 ** fixed.Q_T / 2 ** fixed.S_COL)
        assert abs(complex(int(Zr[k, l]), int(Zi[k, l])) - ex) <= bound, (k, l)
    # against the FP64 DFT with exact twiddles, at scale 2^6
    ref = np.fft.fft2(np.pad((zr + 1j * zi).astype(np.complex128), ((0, 64 - M), (0, 64 - N)))) / 2.0 ** 9
    err = np.abs((Zr + 1j * Zi) - ref)
    assert err.max() <= 2e-4 * np.abs(ref).max(), err.max() / np.abs(ref).max()


def test_fixed_split_and_coefficient_scales():
    """R2 / 2^7 is the FP64 oracle's R_w and W2 / 2^14 its W (eq. (7) on
    the same area), and the first coefficient c / 2^16 is gamma R_w / W0,
    each within the quantisation of the encoding."""
    from oracle import fixed
    s, A = _fixed_area(seed=6)
    M, N = s.shape
    wq = np.where(A, fixed.window_q(M, N, 0.8), 0)
    Zr, Zi = fixed.transform(s * wq, wq << fixed.IMAG_SHIFT)
    Rx, Ry, Wx, Wy = fixed.split(Zr, Zi)
    w = wq / 2.0 ** fixed.Q_W
    EM, EN = cfse.analysis_matrix(64, M), cfse.analysis_matrix(64, N)
    R = cfse.project(w * s + 0j, EM, EN)
    Wf = cfse.project(w + 0j, EM, EN)
    assert np.abs((Rx + 1j * Ry) / 2.0 ** 7 - R).max() <= 2e-4 * np.abs(R).max()
    assert np.abs((Wx + 1j * Wy) / 2.0 ** 14 - Wf).max() <= 2e-4 * np.abs(Wf).max()
    res = fixed.cfse_fixed(s, wq, 0.5, 1)
    u, v = divmod(res["seq"][0], 64)
    c = complex(*res["c"][0]) / 2.0 ** fixed.Q_C
    assert abs(c - 0.5 * R[u, v] / Wf[0, 0].real) <= 1e-4 * abs(R).max() / Wf[0, 0].real


def test_fixed_follows_the_fp64_oracle():
    """Along the FP64 oracle's selections, the fixed-point coefficients stay
    within 2e-3 px of the FP64 ones over 300 iterations (no growth of the
    error: the loop has no division) and the model on B within 0.1 px; free
    running, the two choose the same bins until a near tie."""
    from oracle import fixed
    frames = synth.synthetic_frames(96, 96, (12,))
    blk = np.zeros(1, dtype=synth.BLOCK_DTYPE)[0]
    blk["y0"], blk["x0"], blk["bh"], blk["bw"], blk["border"], blk["fft"], blk["iters"] = 40, 40, 16, 16, 16, 64, 300
    av = np.ones_like(frames)
    av[0, 40:56, 40:56] = 0
    dist = frames * av
    ro = cfse.extrapolate_block(dist, av, blk, 0.8, 0.5)
    rf = fixed.extrapolate_block(dist, av, blk, 0.8, 0.5, forced=ro["seq"])
    err = np.abs(np.array([complex(*c) for c in rf["c"]]) / 2.0 ** fixed.Q_C - np.array(ro["chat"]))
    assert err.max() <= 2e-3, err.max()
    assert err[200:].max() <= 2 * err[:100].max() + 1e-3
    assert np.abs(rf["values"] - ro["values"]).max() <= 0.1
    free = fixed.extrapolate_block(dist, av, blk, 0.8, 0.5, iters=60)
    gap = np.array(ro["gap"][:60])
    first_tie = int(np.argmax(gap < 1e-3)) if (gap < 1e-3).any() else 60
    assert free["seq"][:first_tie] == ro["seq"][:first_tie]


def test_fixed_constant_area_and_bounds():
    """A constant area selects DC every iteration and is reproduced as
    77 (1 - (1 - gamma)^I) to the output step 2^-8; with all pixels 255 on
    a full 64 x 64 support every stored value fits int32 and every product
    int64 (the encoding's range)."""
    from oracle import fixed
    M = N = 48
    A = np.ones((M, N), dtype=bool)
    A[16:32, 16:32] = False
    wq = np.where(A, fixed.window_q(M, N, 0.8), 0)
    res = fixed.cfse_fixed(np.where(A, 77, 0), wq, 0.5, 6)
    assert res["seq"] == [0] * 6
    assert np.abs(res["out"][16:32, 16:32] - 77 * (1 - 0.5 ** 6)).max() <= 2.0 ** -7
    wq = fixed.window_q(64, 64, 1.0)
    zr, zi = 255 * wq, wq << fixed.IMAG_SHIFT
    Zr, Zi = fixed.transform(zr, zi)
    Rx, Ry, Wx, Wy = fixed.split(Zr, Zi)
    lim = 2 ** 31
    for a in (Zr, Zi, Rx, Ry, Wx, Wy):
        assert np.abs(a).max() < lim
    G = (fixed.gamma_q(1.0) << 33) // int(Wx[0, 0])
    assert abs(int(np.abs(Rx).max()) * G) < 2 ** 62
    assert abs(fixed.rshift(int(np.abs(Rx).max()) * G, fixed.S_G)) < 2 ** 24   # coefficients exact in FP32


def test_3d_candidate_restriction():
    """The 3-D candidate mask restricts the dictionary only: all-true equals
    the unrestricted run; a mask of (k, l) columns keeps every selection in
    it with monotone energy; a single candidate is selected every time."""
    from oracle import cfse3
    rng = np.random.default_rng(14)
    M, N, T, F, Ft = 10, 10, 4, 16, 8
    s = rng.normal(size=(M, N, T)) * 20 + 100
    A = rng.random((M, N, T)) > 0.2
    w = np.where(A, cfse3.window(M, N, T, 0.8), 0.0)
    sA = np.where(A, s, 0)
    full = cfse3.cfse3(sA, w, F, Ft, 0.5, 10)
    allc = cfse3.cfse3(sA, w, F, Ft, 0.5, 10, cand=np.ones((F, F, Ft), bool))
    assert full["seq"] == allc["seq"] and np.allclose(full["chat"], allc["chat"], rtol=0, atol=0)
    cols = np.zeros((F, F), bool)
    cols[rng.choice(F, 6), rng.choice(F, 6)] = True
    cand = np.repeat(cols[:, :, None], Ft, axis=2)
    r = cfse3.cfse3(sA, w, F, Ft, 0.5, 12, cand=cand)
    assert all(cand.ravel()[i] for i in r["seq"])
    assert all(b <= a * (1 + 1e-12) for a, b in zip(r["energy"], r["energy"][1:]))
    one = np.zeros((F, F, Ft), bool)
    one[3, 5, 2] = True
    r1 = cfse3.cfse3(sA, w, F, Ft, 0.5, 4, cand=one)
    assert r1["seq"] == [(3 * F + 5) * Ft + 2] * 4
