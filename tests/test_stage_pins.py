"""Pins of the fast summation's stages (Section 3: the kernel replaced by a
trigonometric polynomial, evaluated by an adjoint NFFT, a multiplication by
its coefficients and an NFFT) on the CPU, through the library's host-only
entry points anova_kaiser_bessel and anova_axis_coefficients:

  * the Kaiser-Bessel window against its Fourier transform by quadrature;
  * the coefficients b_k against the Gaussian's Fourier transform (textbook
    closed form) where no regularisation is active, and the trigonometric
    interpolant against the Gaussian on the box;
  * one axis of spread, grid step (the library's circulant column) and gather,
    written out with numpy, against the direct trigonometric-polynomial sum
    sum_k b_k c_k e^{2 pi i k x_j}, c_k = sum_i v_i e^{-2 pi i k x_i} (NDFT).
No GPU is needed."""
import os

import numpy as np
import pytest

import paper_2312_00538_amd as lib


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lib.LIB_PATH):
        from paper_2312_00538_amd import build
        build.build(verbose=False)
    return lib.load_library()


@pytest.mark.parametrize("m,os_", [(2, 2), (3, 2), (4, 2), (4, 3)])
def test_kaiser_bessel_pair_by_quadrature(L, m, os_):
    # The window phi(u) = sinh(b s)/(pi s), s = sqrt(m^2 - u^2), on [-m, m] has
    # the transform I0(m sqrt(b^2 - w^2)) of the NFFT literature up to a term of
    # the size 2 / (pi m b) (the exact transform of the sinh form is a Struve
    # function; the difference is nearly the same for every frequency). The
    # integrand is analytic in u (a function of s^2), so Gauss-Legendre
    # quadrature converges to machine precision.
    o = lib.default_opts(cutoff_m=m, oversample=os_)
    n = os_ * o.n_bw
    b = np.pi * (2.0 - o.n_bw / n)
    v0 = np.sinh(b * m) / (np.pi * m)               # phi(0): the library normalises by it
    xg, wg = np.polynomial.legendre.leggauss(600)
    u = m * xg
    phi, phat = lib.kaiser_bessel(u, o)
    # the window itself: even, 1 at the centre, the closed form at every node
    s = np.sqrt(m * m - u * u)
    assert np.allclose(phi, np.sinh(b * s) / (np.pi * s) / v0, rtol=1e-13, atol=0)
    assert np.allclose(phi, phi[::-1], rtol=1e-13)
    k = np.arange(n // 2 + 1)
    quad = m * (wg[None, :] * phi[None, :] * np.cos(2 * np.pi * k[:, None] * u[None, :] / n)).sum(axis=1)
    diff = quad - n * phat
    bound = 2.0 / (np.pi * m * b) / v0
    print(f"m={m} os={os_}: max |quad - n phi_hat| = {np.abs(diff).max():.2e} (bound {bound:.2e}, "
          f"phi_hat(0) n = {n * phat[0]:.4f}); spread of the difference {np.ptp(diff):.1e}")
    assert np.abs(diff).max() <= 1.1 * bound
    assert np.abs(diff).max() <= 1e-4 * n * phat[0]
    # the transform is positive over the bandwidth and decays past it
    assert np.all(phat[: o.n_bw // 2 + 1] > 0)


def test_coefficients_equal_the_gaussian_transform_without_regularisation(L):
    # sigma_a = 0.04 in torus units: the Gaussian and its first derivative are
    # below 1e-15 where the regularisation takes over (|t| >= 1/2 - eps_b =
    # 1/4), and its spectrum is below 1e-16 at the Nyquist frequency of
    # n_bw = 96, so with the lowest-order bridge (p = 2) the interpolation
    # coefficients are the textbook transform sqrt(pi) sigma exp(-pi^2 sigma^2 k^2)
    # to rounding; the automatic choice of p (a higher-order bridge, matching
    # more derivatives) moves them by less than 1e-8
    k = np.arange(-48, 48)
    for reg_p, tol in ((2, 1e-12), (0, 1e-8)):
        o = lib.default_opts(n_bw=96, reg_p=reg_p)
        c = lib.axis_coefficients(-1.0, 1.0, 0.32, o)
        sa = c["sigma_a"]
        assert abs(sa - 0.04) < 1e-15
        ref = np.sqrt(np.pi) * sa * np.exp(-(np.pi * sa * k) ** 2)
        err = np.abs(c["bk"] - ref).max()
        print(f"reg_p {c['reg_p']}: max |b_k - transform| = {err:.2e} (b_0 = {ref[48]:.4f})")
        assert err <= tol * ref[48]


@pytest.mark.parametrize("lo,hi,sigma,bound", [(-0.25, 0.25, 1.0, 1e-8), (-0.25, 0.25, 0.25, 1e-8),
                                               (-3.0, 5.0, 16.0, 1e-8), (0.0, 1.0, 4.0, 1e-8),
                                               (-3.0, 5.0, 1.7, 1e-3)])
def test_interpolant_reproduces_the_gaussian_on_the_box(L, lo, hi, sigma, bound):
    # sum_k b_k e^{2 pi i k t} (the unpaired -n_bw/2 term as a cosine) against
    # exp(-t^2/sigma_a^2) on a dense grid of the box |t| <= 1/2 - eps_b: the
    # largest difference is what the library reports, and below 1e-8 for the
    # workloads' widths (sigma >= 0.25 on data scaled into [-1/4, 1/4]); the last
    # case (unscaled data, sigma_a = 0.053) is too narrow for bandwidth 32 and
    # reports an error near 1e-4, which is what the request server rejects
    o = lib.default_opts()
    c = lib.axis_coefficients(lo, hi, sigma, o)
    nb = o.n_bw
    t = np.linspace(-(0.5 - o.eps_b), 0.5 - o.eps_b, 4001)
    k = np.arange(-nb // 2, nb // 2)
    terms = c["bk"][None, :] * np.cos(2 * np.pi * k[None, :] * t[:, None])
    val = terms.sum(axis=1)
    err = np.abs(val - np.exp(-(t / c["sigma_a"]) ** 2)).max()
    # map: the data range lands on the box
    assert abs((lo - c["center"]) * c["scale"] + (0.5 - o.eps_b) / 2) < 1e-14
    assert abs((hi - c["center"]) * c["scale"] - (0.5 - o.eps_b) / 2) < 1e-14
    print(f"range [{lo}, {hi}] sigma {sigma}: sigma_a {c['sigma_a']:.4f} p {c['reg_p']} max error {err:.2e} "
          f"(reported {c['kerr']:.2e})")
    assert err <= 1.05 * c["kerr"] + 1e-15
    assert c["kerr"] <= bound


@pytest.mark.parametrize("m,os_,tol", [(4, 2, 2e-7), (3, 2, 1e-5), (4, 3, 2e-8)])
def test_one_axis_spread_grid_step_gather_equals_the_trig_sum(L, m, os_, tol):
    # One feature (a one-dimensional window): spread with the library's window
    # values, circular convolution with its circulant column, gather with the
    # window, against the direct trigonometric-polynomial sum with its b_k.
    # The difference is the NFFT window error alone (the kernel approximation
    # error is common to both sides).
    o = lib.default_opts(cutoff_m=m, oversample=os_)
    n, nb = os_ * o.n_bw, o.n_bw
    rng = np.random.default_rng(2)
    x = rng.uniform(-1.0, 2.0, 300)
    v = rng.standard_normal(300)
    c = lib.axis_coefficients(x.min(), x.max(), 0.9, o)
    u = (x - c["center"]) * c["scale"]                 # torus coordinates in the box
    nu = n * u
    fl = np.floor(nu)
    q = fl.astype(int) - m + 1                          # first of the 2m cells
    offs = (nu - fl)[:, None] + (m - 1 - np.arange(2 * m))[None, :]   # nu - (q + a)
    w, _ = lib.kaiser_bessel(offs.reshape(-1), o)
    w = w.reshape(-1, 2 * m)
    cells = (q[:, None] + np.arange(2 * m)[None, :]) % n
    g = np.zeros(n)
    np.add.at(g, cells, v[:, None] * w)                 # spread
    circ = c["circ"]
    idx = (np.arange(n)[:, None] - np.arange(n)[None, :]) % n
    h = circ[idx] @ g                                   # h_l = sum_d circ[l - d] g_d
    f = (h[cells] * w).sum(axis=1)                      # gather
    k = np.arange(-nb // 2, nb // 2)
    ck = (v[None, :] * np.exp(-2j * np.pi * k[:, None] * u[None, :])).sum(axis=1)
    bk = c["bk"].copy()
    # the unpaired frequency -n_bw/2 enters as a cosine: half at -n_bw/2, half at +n_bw/2
    trig = (bk[:, None] * ck[:, None] * np.exp(2j * np.pi * k[:, None] * u[None, :])).sum(axis=0)
    trig += -0.5 * bk[0] * ck[0] * np.exp(2j * np.pi * k[0] * u) \
        + 0.5 * bk[0] * np.conj(ck[0]) * np.exp(-2j * np.pi * k[0] * u)
    ref = trig.real
    err = np.linalg.norm(f - ref) / np.linalg.norm(ref)
    gauss = np.exp(-((u[:, None] - u[None, :]) / c["sigma_a"]) ** 2) @ v
    egauss = np.linalg.norm(f - gauss) / np.linalg.norm(gauss)
    print(f"m={m} os={os_}: NFFT vs trigonometric sum {err:.2e}; vs the Gaussian sum {egauss:.2e}")
    assert err <= tol
    # against the Gaussian itself the kernel approximation error adds in (its
    # largest pointwise value here is c["kerr"], ~1e-9)
    assert egauss <= max(tol, 1e-7)
