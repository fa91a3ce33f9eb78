"""The split's factorisation on its own (gcamps_factorize: Gram on MFMA, block-Jacobi eigensolver,
truncation rule, emit) against LAPACK singular values and the oracle's truncation rule, from
1 x 7 up to the library's maximum matrix side, 4096 (a ctx with chi_max = 2048 and d = 2): there
the eigensolver runs 128 sub-problems per round, each rebuilt from the matrix before the previous
round's update while that update runs in the same launch.

Bars.  With sigma_0 the largest singular value:
- kept rank equals the oracle's rule on the LAPACK values (the cases are built with no value
  near a decision threshold);
- every sigma_i^2 within 1e-11 sigma_0^2 of LAPACK's: the FP64 Gram (sums of up to 4096
  products) and the Jacobi rotations fix its eigenvalues to a small multiple of
  m * eps * sigma_0^2, and 1e-11 is 22 m eps at m = 4096 (measured: 1.7e-12 there);
  the kept values within 1e-12 sigma_0;
- discarded weight within 1e-9 relative (1e-12 absolute);
- factors: L has orthonormal columns (1e-12) and R = L^dagger M / |s_k| (1e-10 of the largest
  entry), which with the first bar makes L R the normalised rank-k truncation of M.
With cutoff 0 the rank floor decides, through the relative-accuracy second pass: an exactly
rank-50 matrix keeps 50 with its null values below the floor, and a graded spectrum
sigma_i = 10^(-0.3 i) keeps 44 (values down to 1.3e-13 sigma_0), checked against the
constructed spectrum itself.

The rank-reduced path (GCAMPS_FACTORIZE_REDUCE, used for the splits after a disentangler) is held
to the same bars: a pivoted Cholesky factorisation of the Gram stops once the remaining trace is
below min(1e-14, cutoff / 2m) of the whole, so every singular value it leaves out has
sigma^2 <= 5.6e-14 sigma_0^2 m here, inside the 1e-11 sigma_0^2 bar, and the remainder is counted
as discarded weight (inside the 1e-12 absolute bar); it applies for 320 < min(p, q) <= 1024.  Cases: exact rank m/3 (the shape of a
rotated two-site tensor at chi = 256: 768 x 768, rank 256), rank plus noise below the bound, a
decaying spectrum cut by the cutoff inside the reduced basis, a full-rank matrix, where every
row is pivoted and the complement is empty, and with chi_max = 256: a cut set by the cap, a
degenerate pair at the cap, and a plateau of weak values under the cutoff.
"""
import sys

import numpy as np
import pytest

from oracle.mps import rtrunc, svd

pytestmark = pytest.mark.gpu
CHI, CUT = 2048, 1e-10


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def g():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2511_06672_amd import gcamps
    gcamps.lib()
    return gcamps


def state(g, cutoff, chi=CHI, d=2):
    return g.State(g.make_config(d, 2, chi, cutoff, auto_disentangle=False, max_candidates=1))


def gauss(rng, p, q):
    return (rng.standard_normal((p, q)) + 1j * rng.standard_normal((p, q))) / np.sqrt(2)


def check(g, st, m, cutoff, factors, reduce=False, kept_tol=1e-12, chi=CHI):
    sig, k, eps, L, R = st.factorize(m, factors=factors, reduce=reduce)
    ref = np.linalg.svd(m, compute_uv=False)
    kr, er, _ = rtrunc(ref, cutoff, chi)
    s0 = ref[0]
    assert k == kr
    assert np.all(np.diff(sig) <= 0)
    assert np.max(np.abs(sig[:k] - ref[:k])) <= kept_tol * s0
    assert np.max(np.abs(sig ** 2 - ref ** 2)) <= 1e-11 * s0 ** 2
    assert abs(eps - er) <= max(1e-9 * er, 1e-12)
    if factors:
        assert L.shape == (m.shape[0], k) and R.shape == (k, m.shape[1])
        assert np.max(np.abs(L.conj().T @ L - np.eye(k))) <= 1e-12
        proj = L.conj().T @ m / np.linalg.norm(ref[:k])
        assert np.max(np.abs(R - proj)) <= 1e-10 * np.max(np.abs(proj))
    return k, sig, s0


@pytest.mark.parametrize("p,q", [(1, 7), (7, 1), (5, 3), (33, 70), (70, 33), (300, 97), (1536, 1600)])
def test_factorize_gaussian_shapes(g, p, q):
    say(f"factorize gaussian {p} x {q}")
    st = state(g, CUT)
    rng = np.random.default_rng(1000 + p + 7 * q)
    k, _, _ = check(g, st, gauss(rng, p, q), CUT, factors=True)
    assert k == min(p, q)            # no value falls under the cutoff or the floor


def test_factorize_cutoff_and_rank_floor(g):
    rng = np.random.default_rng(77)
    say("factorize rank 200 plus 1e-9 noise (the cutoff decides), 900 x 1200")
    m = gauss(rng, 900, 200) @ gauss(rng, 200, 1200) / np.sqrt(200) + 1e-9 * gauss(rng, 900, 1200)
    assert check(g, state(g, CUT), m, CUT, factors=True)[0] == 200
    say("factorize exact rank 50, cutoff 0 (the rank floor decides after the second pass), 600 x 600")
    m = gauss(rng, 600, 50) @ gauss(rng, 50, 600)
    k, sig, s0 = check(g, state(g, 0.0), m, 0.0, factors=True)
    assert k == 50 and np.max(sig[50:]) <= 1e-13 * s0


def test_factorize_graded_spectrum_second_pass(g):
    say("factorize graded spectrum 10^(-0.3 i), 128 x 128, cutoff 0")
    st = state(g, 0.0)
    rng = np.random.default_rng(78)
    u, _, _ = svd(gauss(rng, 128, 128))
    v, _, _ = svd(gauss(rng, 128, 128))
    true = 10.0 ** (-0.3 * np.arange(128))
    m = (u * true) @ v.conj().T
    sig, k, eps, L, R = st.factorize(m, factors=True)
    assert k == 44                   # sigma_43 = 10^-12.9 > 1e-13 sigma_0 > sigma_44 = 10^-13.2
    # forming m rounds it by about eps * sqrt(128) sigma_0, which bounds how far its singular
    # values can sit from the constructed ones
    assert np.max(np.abs(sig[:k] - true[:k])) <= 2e-14
    assert np.max(np.abs(L.conj().T @ L - np.eye(k))) <= 1e-12
    assert abs(eps - np.sum(true[k:] ** 2) / np.sum(true ** 2)) <= 1e-15


@pytest.mark.parametrize("p,q,r", [(768, 768, 256), (729, 1458, 243), (1458, 729, 243), (400, 400, 150)])
def test_factorize_reduced_exact_rank(g, p, q, r):
    say(f"factorize reduced, exact rank {r} in {p} x {q}")
    rng = np.random.default_rng(500 + p + q + r)
    m = gauss(rng, p, r) @ gauss(rng, r, q) / np.sqrt(r)
    st = state(g, CUT)
    k, sig, s0 = check(g, st, m, CUT, factors=True, reduce=True)
    assert k == r
    ks = st.kernel_stats()
    assert ks["reduced"] == 1 and ks["reduced_basis_frac"] <= (r + 16) / min(p, q)


def test_factorize_reduced_noise_and_decaying_spectrum(g):
    rng = np.random.default_rng(501)
    say("factorize reduced, rank 200 plus 1e-9 noise, 900 x 1200")
    m = gauss(rng, 900, 200) @ gauss(rng, 200, 1200) / np.sqrt(200) + 1e-9 * gauss(rng, 900, 1200)
    assert check(g, state(g, CUT), m, CUT, factors=True, reduce=True)[0] == 200
    # sigma_i = 10^(-0.047 i): the tail after k values is 10^(-0.094 k), so the cutoff falls
    # between k = 106 (tail 1.1e-10) and k = 107 (0.87e-10), away from either
    say("factorize reduced, sigma_i = 10^(-0.047 i) on 600 x 600 (the cutoff cuts inside the basis)")
    u, _, _ = svd(gauss(rng, 600, 600))
    v, _, _ = svd(gauss(rng, 600, 600))
    true = 10.0 ** (-0.047 * np.arange(600))
    m = (u * true) @ v.conj().T
    ref = np.linalg.svd(m, compute_uv=False)
    # Kept values reach 1e-5 sigma_0 here, where a Gram's absolute eigenvalue error (~1e-16
    # sigma_0^2) is ~1e-11 sigma_0 in sigma: the reduced path must be as accurate as the full one
    full = state(g, CUT)
    sf, kf, _, _, _ = full.factorize(m)
    err_full = np.max(np.abs(sf[:kf] - ref[:kf]))
    st = state(g, CUT)
    k, sig, s0 = check(g, st, m, CUT, factors=True, reduce=True, kept_tol=max(1e-12, 4 * err_full))
    err_red = np.max(np.abs(sig[:k] - ref[:k]))
    say(f"  kept sigma error: reduced {err_red:.2e}, full {err_full:.2e} (sigma_0 = {s0:.3f})")
    assert k == kf == 107
    assert st.kernel_stats()["reduced"] == 1


def test_factorize_reduced_on_full_rank(g):
    say("factorize through the Cholesky path on a full-rank 400 x 500 gaussian (every row pivoted)")
    rng = np.random.default_rng(502)
    st = state(g, CUT)
    k, _, _ = check(g, st, gauss(rng, 400, 500), CUT, factors=True, reduce=True)
    assert k == 400
    ks = st.kernel_stats()
    assert ks["reduced"] == 1 and ks["reduced_basis_frac"] == 1.0


def spectrum_matrix(rng, n, true):
    u, _, _ = svd(gauss(rng, n, n))
    v, _, _ = svd(gauss(rng, n, n))
    return (u * true) @ v.conj().T


def test_factorize_reduced_cut_by_the_cap(g):
    """chi_max = 256 on a 768 x 768 matrix with sigma_i = 10^(-0.012 i), the shape of a rotated
    two-site tensor at chi = 256: the cap sets the cut (the tail after 256 values is 7e-7 of the
    weight, far above the cutoff) inside a basis of ~600 columns."""
    say("factorize reduced, cut by chi_max = 256: sigma_i = 10^(-0.012 i), 768 x 768")
    rng = np.random.default_rng(504)
    m = spectrum_matrix(rng, 768, 10.0 ** (-0.012 * np.arange(768)))
    st = state(g, CUT, chi=256, d=3)
    k, _, _ = check(g, st, m, CUT, factors=True, reduce=True, chi=256)
    assert k == 256 and st.kernel_stats()["reduced"] == 1


def test_factorize_reduced_degenerate_pair_at_the_cap(g):
    """sigma_255 = sigma_256 exactly with chi_max 256: the degeneracy guard moves the cut to 255,
    so that no multiplet is split."""
    say("factorize reduced, degenerate pair at the cap: 768 x 768, chi_max 256")
    rng = np.random.default_rng(506)
    true = 10.0 ** (-0.012 * np.arange(768))
    true[256] = true[255]
    st = state(g, CUT, chi=256, d=3)
    k, _, _ = check(g, st, spectrum_matrix(rng, 768, true), CUT, factors=True, reduce=True, chi=256)
    assert k == 255


def test_factorize_reduced_plateau_under_the_cutoff(g):
    """100 values 10^(-0.02 i) above a plateau of 500 values sigma = 3e-7 (each ~8e-15 of the
    weight, 4e-12 together): the cutoff discards the whole plateau, which the Cholesky
    factorisation must still pivot almost entirely to reach its 1e-14 stop."""
    say("factorize reduced, 100 values above a 500-value plateau, 600 x 600, chi_max 256")
    rng = np.random.default_rng(505)
    true = np.concatenate([10.0 ** (-0.02 * np.arange(100)), np.full(500, 3e-7)])
    st = state(g, CUT, chi=256, d=3)
    k, _, _ = check(g, st, spectrum_matrix(rng, 600, true), CUT, factors=True, reduce=True, chi=256)
    ks = st.kernel_stats()
    assert k == 100 and ks["reduced"] == 1 and ks["reduced_basis_frac"] > 256 / 600


def test_factorize_small_sides_keep_the_plain_path(g):
    say("factorize with the reduce flag at min side 200 (below the Cholesky path's range)")
    rng = np.random.default_rng(503)
    st = state(g, CUT)
    check(g, st, gauss(rng, 200, 50) @ gauss(rng, 50, 300) / np.sqrt(50), CUT, factors=True, reduce=True)
    assert st.kernel_stats()["reduced"] == 0


def test_factorize_maximum_size(g):
    say("factorize gaussian 4096 x 4096 (maximum matrix side; chi_max 2048 keeps half)")
    st = state(g, CUT)
    rng = np.random.default_rng(4096)
    assert check(g, st, gauss(rng, 4096, 4096), CUT, factors=False)[0] == CHI


def test_factorize_errors(g):
    say("factorize error paths")
    st = state(g, CUT)
    with pytest.raises(g.GcampsError) as e:
        st.factorize(np.zeros((4097, 4097)))
    assert e.value.code == -4        # ECAPACITY
    with pytest.raises(g.GcampsError) as e:
        st.factorize(np.zeros((3, 3)))
    assert e.value.code == -6        # ENUMERIC: a zero matrix has nothing to keep
