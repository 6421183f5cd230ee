"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against mathematics the paper's problem statement
fixes (Sec. 2: the exact 3D DFT of a real array and its inverse): closed forms,
the literal definition on tiny inputs, an independent library (numpy's
pocketfft), and invariants (Parseval, Hermitian symmetry, linearity, shift,
round trip).  A dropped term, a wrong sign or index, or a transposed operand in
the oracle fails at least one of them.
"""
import numpy as np
import pytest

from workloads import fields

pytestmark = []


def all_23_smooth(limit):
    out = []
    p2 = 1
    while p2 <= limit:
        p3 = p2
        while p3 <= limit:
            out.append(p3)
            p3 *= 3
        p2 *= 2
    return sorted(out)


# Every 2^a 3^b length up to 1024, lengths with factors 5 and 7 (the GPU
# path's radix-5/7 stages), and a few with other primes: the oracle itself
# accepts any n.
LENGTHS = all_23_smooth(1024) + [5, 7, 10, 11, 13, 15, 25, 35, 49, 97, 125, 175, 245, 343, 625, 2401]


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# ----------------------------------------------------------------- 1D ----

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8, 12, 16])
def test_dft1d_closed_forms(oracle, n):
    k = np.arange(n)
    # delta at a: X[k] = e^{-2 pi i k a / n}
    for a in range(n):
        x = np.zeros(n, complex)
        x[a] = 1.0
        X = oracle.dft1d(x, -1)
        assert np.max(np.abs(X - np.exp(-2j * np.pi * ((k * a) % n) / n))) < 4e-15
    # constant: n at k = 0 only
    X = oracle.dft1d(np.full(n, 2.5 + 0j), -1)
    expect = np.zeros(n, complex)
    expect[0] = 2.5 * n
    assert np.max(np.abs(X - expect)) < 1e-13
    # e^{+2 pi i m j / n}: the forward (minus) transform peaks at +m
    for m in range(n):
        x = np.exp(2j * np.pi * m * k / n)
        X = oracle.dft1d(x, -1)
        expect = np.zeros(n, complex)
        expect[m] = n
        assert np.max(np.abs(X - expect)) < 1e-12
        # and the plus-sign transform of the same input peaks at -m
        Xp = oracle.dft1d(x, +1)
        expect = np.zeros(n, complex)
        expect[(-m) % n] = n
        assert np.max(np.abs(Xp - expect)) < 1e-12


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 27, 60, 128])
def test_dft1d_matches_numpy(oracle, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert rel(oracle.dft1d(x, -1), np.fft.fft(x)) < 1e-14
    assert rel(oracle.dft1d(x, +1), np.fft.ifft(x) * n) < 1e-14


def test_fft1d_matches_naive_at_every_length(oracle):
    rng = np.random.default_rng(7)
    worst = 0.0
    for n in LENGTHS:
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        for sign in (-1, +1):
            r = rel(oracle.fft1d(x, sign), oracle.dft1d(x, sign))
            worst = max(worst, r)
            assert r < 1e-14, (n, sign, r)
    # expected accuracy ~ eps * sqrt(log n)
    assert worst < 2e-15


def smooth2357(lo, hi):
    out = []
    for a in range(14):
        for b in range(9):
            for c in range(6):
                for d in range(5):
                    n = 2 ** a * 3 ** b * 5 ** c * 7 ** d
                    if lo < n <= hi:
                        out.append(n)
    return sorted(out)


# Lengths above 1024 at which the GPU tests use the oracle as the reference
# (n2 rows of 1536 .. 8192, n1 columns of 2048 and 4096, n0 columns of 4096,
# radix-5/7 lines of 1400 and 2401): every 2^a 3^b 5^c 7^d length in
# (1024, 8192] against numpy's pocketfft, an independent library.
LONG = smooth2357(1024, 8192)


def test_fft1d_matches_numpy_at_long_lengths(oracle):
    rng = np.random.default_rng(8)
    worst = 0.0
    for n in LONG:
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        r = rel(oracle.fft1d(x, -1), np.fft.fft(x))
        ri = rel(oracle.fft1d(x, +1), np.fft.ifft(x) * n)
        worst = max(worst, r, ri)
        assert r < 1e-14 and ri < 1e-14, (n, r, ri)
    assert worst < 4e-15


@pytest.mark.slow
@pytest.mark.parametrize("n", [1400, 1536, 2048, 3072, 4096, 8192])
def test_fft1d_matches_naive_at_long_lengths(oracle, n):
    # the definition itself (O(n^2), long double), at the long lengths the
    # GPU tests feed the oracle
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for sign in (-1, +1):
        r = rel(oracle.fft1d(x, sign), oracle.dft1d(x, sign))
        assert r < 1e-14, (n, sign, r)


def test_fft1d_rejects_bad_args(oracle):
    with pytest.raises(RuntimeError):
        oracle.fft1d(np.zeros(0, complex))


# --------------------------------------------------- 3D, definition ----

TINY = [(1, 1, 1), (1, 1, 2), (2, 3, 5), (3, 5, 7), (4, 6, 8), (8, 8, 8), (5, 1, 2), (1, 4, 6),
        (2, 2, 3), (6, 4, 1)]


@pytest.mark.parametrize("shape", TINY)
def test_r2c_matches_triple_sum(oracle, shape):
    x = fields.uniform(shape, seed=11)
    X = oracle.r2c(x)
    Xd = oracle.r2c_direct(x)
    assert X.shape == (shape[0], shape[1], shape[2] // 2 + 1)
    assert rel(X, Xd) < 1e-14


@pytest.mark.parametrize("shape", TINY)
def test_c2r_matches_definition_on_arbitrary_spectrum(oracle, shape):
    # a random, non-Hermitian half spectrum: checks the DC/Nyquist reading too
    rng = np.random.default_rng(12)
    h = shape[2] // 2 + 1
    X = rng.standard_normal((shape[0], shape[1], h)) + 1j * rng.standard_normal((shape[0], shape[1], h))
    y, max_im = oracle.c2r(X, shape[2], return_max_imag=True)
    yd = oracle.c2r_direct(X, shape[2])
    assert rel(y, yd) < 1e-14
    assert max_im < 1e-12 * max(1.0, np.abs(y).max())


@pytest.mark.parametrize("shape", [(4, 6, 8), (3, 5, 7), (8, 8, 8), (2, 4, 2)])
def test_point_values_match_definition(oracle, shape):
    x = fields.uniform(shape, seed=13)
    Xd = oracle.r2c_direct(x)
    rng = np.random.default_rng(14)
    h = shape[2] // 2 + 1
    S = rng.standard_normal((shape[0], shape[1], h)) + 1j * rng.standard_normal((shape[0], shape[1], h))
    yd = oracle.c2r_direct(S, shape[2])
    for k0 in range(shape[0]):
        for k1 in range(shape[1]):
            for k2 in range(h):
                assert abs(oracle.r2c_point(x, (k0, k1, k2)) - Xd[k0, k1, k2]) < 1e-12
    for j in [(0, 0, 0), (shape[0] - 1, shape[1] - 1, shape[2] - 1), (1 % shape[0], 2 % shape[1], 3 % shape[2])]:
        assert abs(oracle.c2r_point(S, shape[2], j) - yd[j]) < 1e-12


def test_point_values_match_numpy_at_64(oracle):
    shape = (64, 48, 40)
    x = fields.uniform(shape, seed=15)
    Xn = np.fft.rfftn(x)
    S = fields.k53_spectrum(shape, seed=16)
    yn = np.fft.irfftn(S, s=shape, axes=(0, 1, 2), norm="forward")
    for k in [(0, 0, 0), (63, 47, 20), (5, 41, 7), (32, 24, 0), (1, 0, 20)]:
        assert abs(oracle.r2c_point(x, k) - Xn[k]) < 1e-9
    for j in [(0, 0, 0), (63, 47, 39), (10, 3, 17)]:
        assert abs(oracle.c2r_point(S, 40, j) - yn[j]) < 1e-11


# ------------------------------------------------ independent library ----

@pytest.mark.parametrize("shape", [(32, 32, 32), (64, 48, 40), (96, 32, 64), (27, 12, 18), (16, 16, 9),
                                   (48, 48, 48), (128, 128, 128), (35, 49, 50), (25, 14, 45)])
def test_r2c_c2r_match_pocketfft(oracle, shape):
    x = fields.uniform(shape, seed=17)
    X = oracle.r2c(x)
    assert rel(X, np.fft.rfftn(x)) < 1e-14
    rng = np.random.default_rng(18)
    S = X + 0.1 * (rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape))
    y = oracle.c2r(S, shape[2])
    yn = np.fft.irfftn(S, s=shape, axes=(0, 1, 2), norm="forward")
    assert rel(y, yn) < 1e-14


@pytest.mark.slow
def test_r2c_c2r_match_pocketfft_256(oracle):
    shape = (256, 256, 256)
    x = fields.k53_field(shape, seed=2, kmax=85)
    X = oracle.r2c(x)
    assert rel(X, np.fft.rfftn(x)) < 1e-13
    y = oracle.c2r(X, 256)
    assert rel(y, x * x.size) < 1e-13


# ------------------------------------------------------- closed forms ----

SHAPE = (8, 12, 16)


def _grid(shape):
    return np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")


@pytest.mark.parametrize("m", [(1, 2, 3), (3, 1, 5), (7, 11, 1), (2, 5, 7), (-3, 4, 2)])
def test_single_mode_interior(oracle, m):
    # 0 < m2 < n2/2: cos gives N/2 at (m0 mod n0, m1 mod n1, m2), sin gives -iN/2
    n0, n1, n2 = SHAPE
    N = n0 * n1 * n2
    j0, j1, j2 = _grid(SHAPE)
    th = 2 * np.pi * (m[0] * j0 / n0 + m[1] * j1 / n1 + m[2] * j2 / n2)
    for fn, val in ((np.cos, N / 2), (np.sin, -1j * N / 2)):
        X = oracle.r2c(fn(th))
        expect = np.zeros_like(X)
        expect[m[0] % n0, m[1] % n1, m[2]] = val
        assert np.max(np.abs(X - expect)) < 1e-11 * N


@pytest.mark.parametrize("m", [(1, 2, 0), (3, 5, 0), (0, 0, 8), (2, 3, 8), (4, 6, 8), (4, 0, 0)])
def test_single_mode_self_conjugate_planes(oracle, m):
    # m2 = 0 or n2/2: the mirror (-m0, -m1, m2) is in the stored half too
    n0, n1, n2 = SHAPE
    N = n0 * n1 * n2
    j0, j1, j2 = _grid(SHAPE)
    th = 2 * np.pi * (m[0] * j0 / n0 + m[1] * j1 / n1 + m[2] * j2 / n2)
    a = (m[0] % n0, m[1] % n1, m[2])
    b = ((-m[0]) % n0, (-m[1]) % n1, m[2])
    X = oracle.r2c(np.cos(th))
    expect = np.zeros_like(X)
    expect[a] += N / 2
    expect[b] += N / 2
    assert np.max(np.abs(X - expect)) < 1e-11 * N
    X = oracle.r2c(np.sin(th))
    expect = np.zeros_like(X)
    expect[a] += -1j * N / 2
    expect[b] += 1j * N / 2
    assert np.max(np.abs(X - expect)) < 1e-11 * N


def test_delta_and_constant(oracle):
    n0, n1, n2 = SHAPE
    N = n0 * n1 * n2
    k0, k1, k2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2 // 2 + 1), indexing="ij")
    for a in [(0, 0, 0), (3, 7, 5), (7, 11, 15)]:
        x = np.zeros(SHAPE)
        x[a] = 1.0
        X = oracle.r2c(x)
        # phase k.a/n as an exact integer fraction over N, reduced before exp
        e = (k0 * a[0] * n1 * n2 + k1 * a[1] * n0 * n2 + k2 * a[2] * n0 * n1) % N
        expect = np.exp(-2j * np.pi * e / N)
        assert np.max(np.abs(X - expect)) < 1e-14
    X = oracle.r2c(np.full(SHAPE, -0.75))
    expect = np.zeros_like(X)
    expect[0, 0, 0] = -0.75 * N
    assert np.max(np.abs(X - expect)) < 1e-12


def test_shift_theorem(oracle):
    shape = (12, 8, 18)
    x = fields.uniform(shape, seed=19)
    s = (5, 3, 7)
    X = oracle.r2c(x)
    Xs = oracle.r2c(np.roll(x, s, axis=(0, 1, 2)))
    k0, k1, k2 = np.meshgrid(*[np.arange(n) for n in shape[:2]], np.arange(shape[2] // 2 + 1), indexing="ij")
    n0, n1, n2 = shape
    N = n0 * n1 * n2
    e = (k0 * s[0] * n1 * n2 + k1 * s[1] * n0 * n2 + k2 * s[2] * n0 * n1) % N
    ph = np.exp(-2j * np.pi * e / N)
    assert rel(Xs, ph * X) < 1e-14


@pytest.mark.parametrize("shape", [(8, 12, 16), (9, 6, 10), (5, 7, 9)])
def test_parseval_hermitian_linearity(oracle, shape):
    n0, n1, n2 = shape
    N = n0 * n1 * n2
    x = fields.uniform(shape, seed=20)
    z = fields.uniform(shape, seed=21)
    X = oracle.r2c(x)
    w = np.full(n2 // 2 + 1, 2.0)
    w[0] = 1.0
    if n2 % 2 == 0:
        w[n2 // 2] = 1.0
    lhs = np.sum(x * x)
    rhs = np.sum(w * np.abs(X) ** 2) / N
    assert abs(lhs - rhs) < 1e-12 * lhs
    # Hermitian symmetry of the self-conjugate planes
    planes = [0] + ([n2 // 2] if n2 % 2 == 0 else [])
    for k2 in planes:
        P = X[:, :, k2]
        mirror = np.conj(P[(-np.arange(n0)) % n0][:, (-np.arange(n1)) % n1])
        assert np.max(np.abs(P - mirror)) < 1e-12 * N
    # linearity
    a, b = 0.3, -1.7
    assert rel(oracle.r2c(a * x + b * z), a * X + b * oracle.r2c(z)) < 1e-14


@pytest.mark.parametrize("shape", [(32, 32, 32), (3, 5, 8), (16, 1, 2), (1, 1, 10), (7, 9, 11)])
def test_round_trip(oracle, shape):
    x = fields.uniform(shape, seed=1)
    y = oracle.c2r(oracle.r2c(x), shape[2])
    assert rel(y, x * np.prod(shape)) < 1e-14


def test_c2r_drops_imag_of_self_conjugate_bins(oracle):
    # Im of the (0,0,0) and (0,0,n2/2) bins cannot reach the real output
    shape = (6, 8, 10)
    x = fields.uniform(shape, seed=22)
    X = oracle.r2c(x)
    y = oracle.c2r(X, 10)
    X2 = X.copy()
    X2[0, 0, 0] += 3j
    X2[0, 0, 5] -= 2j
    assert np.max(np.abs(oracle.c2r(X2, 10) - y)) < 1e-12
    # but Im of an off-axis k2 = 0 bin does (non-Hermitian input, definition)
    X3 = X.copy()
    X3[1, 2, 0] += 1j
    assert np.max(np.abs(oracle.c2r(X3, 10) - y)) > 0.1


def test_reduces_to_lower_dimensions(oracle):
    # n0 = 1: the plane step alone, a 2D rfft2; n0 = n1 = 1: a 1D rfft
    x2 = fields.uniform((1, 12, 18), seed=23)
    assert rel(oracle.r2c(x2)[0], np.fft.rfft2(x2[0])) < 1e-14
    x1 = fields.uniform((1, 1, 30), seed=24)
    assert rel(oracle.r2c(x1)[0, 0], np.fft.rfft(x1[0, 0])) < 1e-14
    # n1 = 1, n2 = 2: the plane step is a sum/difference and step 3 a plain
    # length-n0 DFT of each of the two columns
    x = fields.uniform((12, 1, 2), seed=25)
    X = oracle.r2c(x)
    s = x[:, 0, 0] + x[:, 0, 1]
    d = x[:, 0, 0] - x[:, 0, 1]
    assert rel(X[:, 0, 0], oracle.dft1d(s, -1)) < 1e-14
    assert rel(X[:, 0, 1], oracle.dft1d(d, -1)) < 1e-14


def test_natural_order_not_transposed(oracle):
    # distinct extents and a mode with m0 != m1 != m2: a transposed output
    # (n1 x n0 x H) would put the peak elsewhere or fail the shape
    shape = (6, 10, 14)
    j0, j1, j2 = _grid(shape)
    m = (1, 3, 4)
    x = np.cos(2 * np.pi * (m[0] * j0 / 6 + m[1] * j1 / 10 + m[2] * j2 / 14))
    X = oracle.r2c(x)
    assert X.shape == (6, 10, 8)
    flat = np.argmax(np.abs(X).ravel())
    assert flat == (m[0] * 10 + m[1]) * 8 + m[2]


# ------------------------------------------------------ generators ----

def test_velocity_field_is_solenoidal_in_oracle_index_map(oracle):
    shape = (24, 16, 20)
    u = fields.velocity_field(shape, seed=26)
    U = [oracle.r2c(u[c]) for c in range(3)]
    k0 = fields.signed_wavenumbers(24)[:, None, None]
    k1 = fields.signed_wavenumbers(16)[None, :, None]
    k2 = np.arange(11)[None, None, :]
    div = k0 * U[0] + k1 * U[1] + k2 * U[2]
    scale = max(np.abs(U[c]).max() for c in range(3))
    assert np.max(np.abs(div)) < 1e-12 * scale * 24
    assert abs(np.mean(u * u) - 1.0) < 1e-12


def test_k53_field_spectrum_recovered(oracle):
    shape = (32, 24, 40)
    S = fields.k53_spectrum(shape, seed=27)
    x = fields.k53_field(shape, seed=27)
    assert abs(np.sqrt(np.mean(x * x)) - 1.0) < 1e-12
    assert abs(np.mean(x)) < 1e-12
    X = oracle.r2c(x)
    # x = c * irfftn(S), so r2c(x) = c * N * S... up to the normalisation of irfftn
    # (norm="forward" is the plain sum), so r2c(x) = c * N * S with c = 1/rms
    ratio = X[np.abs(S) > 0] / S[np.abs(S) > 0]
    assert np.std(ratio) / abs(np.mean(ratio)) < 1e-12
    assert np.all(np.abs(X[np.abs(S) == 0]) < 1e-9 * np.abs(X).max())
    kmax = fields.default_kmax(shape)
    k0 = fields.signed_wavenumbers(32)[:, None, None]
    k1 = fields.signed_wavenumbers(24)[None, :, None]
    k2 = np.arange(21)[None, None, :]
    kk = np.sqrt(k0 ** 2 + k1 ** 2 + k2 ** 2)
    assert np.all(np.abs(X[kk > kmax]) < 1e-9 * np.abs(X).max())


# ------------------------------------------------------------ pruned --

@pytest.mark.parametrize("shape,kmax", [((12, 10, 16), (4, 3, 5)), ((9, 8, 6), (2, -1, 1)), ((8, 8, 8), (-1, -1, -1)),
                                        ((6, 7, 10), (0, 0, 0))])
def test_box_mask_counts(oracle, shape, kmax):
    """Closed-form size of the box: (2K0+1)(2K1+1)(K2+1), a whole axis for K < 0."""
    n0, n1, n2 = shape
    K0, K1, K2 = kmax
    want = (n0 if K0 < 0 else 2 * K0 + 1) * (n1 if K1 < 0 else 2 * K1 + 1) * (n2 // 2 + 1 if K2 < 0 else K2 + 1)
    assert int(oracle.box_mask(shape, kmax).sum()) == want


def test_pruned_pair_keeps_exactly_the_box_cosines(oracle):
    """A field made of single cosines, some with wavevectors on the edge of
    the box (kept) and some one step beyond it (dropped), including negative
    k0/k1 and the k2 = 0 plane: the pruned inverse of the forward transform
    is N times the sum of the kept cosines alone, evaluated directly."""
    shape = (18, 16, 20)
    n0, n1, n2 = shape
    kmax = (5, 4, 6)
    j0, j1, j2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    waves = [((5, -4, 6), True), ((-5, 4, 0), True), ((0, 0, 0), True), ((3, 1, 2), True),
             ((6, 0, 1), False), ((0, -5, 3), False), ((1, 2, 7), False), ((-6, 4, 0), False)]
    rng = np.random.default_rng(8)
    x = np.zeros(shape)
    kept = np.zeros(shape)
    for (k0, k1, k2), inside in waves:
        a, ph = 1.0 + rng.random(), 2 * np.pi * rng.random()
        term = a * np.cos(2 * np.pi * (k0 * j0 / n0 + k1 * j1 / n1 + k2 * j2 / n2) + ph)
        x += term
        if inside:
            kept += term
    X = oracle.r2c_pruned(x, kmax)
    y = oracle.c2r_pruned(X, n2, kmax) / x.size
    assert rel(y, kept) < 1e-13
    # c2r_pruned also ignores whatever sits outside the box
    Xf = oracle.r2c(x)
    assert rel(oracle.c2r_pruned(Xf, n2, kmax) / x.size, kept) < 1e-13


def test_r2c_pruned_zero_outside_and_exact_inside(oracle):
    shape = (10, 12, 14)
    kmax = (3, 4, 5)
    x = fields.uniform(shape, seed=9)
    X = oracle.r2c_pruned(x, kmax)
    for k in [(3, -4 % 12, 5), (-3 % 10, 4, 0), (0, 0, 0)]:
        want = oracle.r2c_point(x, k)
        assert abs(X[k] - want) <= 1e-12 * abs(want)
    for k in [(4, 0, 0), (0, 5, 1), (0, 12 - 5, 2), (1, 1, 6), (10 - 4, 0, 3)]:
        assert X[k] == 0
