"""GPU parity: every entry point of the HIP path against the FP64 CPU oracle
on the same seeded inputs.  Sizes span several tiles with ragged tails."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import adjoint as ADJ, discretize as D, krylov as KR, precond as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2410_22686_amd import Solver, kkt_solve  # noqa: E402
from parity import check, rel  # noqa: E402

DEV = torch.device("cuda:0")


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def problems(dim, nx, nt, gammas, eps=None, coeff=None):
    return [D.make_problem(dim, nx, nt, gm, eps=eps, coeff=coeff) for gm in gammas]


KKT_CASES = [
    (2, 15, 12, (1e-4,), None),
    (2, 31, 32, (1e-2, 1e-8), None),
    (3, 7, 9, (1e-3,), None),
    (2, 15, 6, (1e-3,), W.coeff_sines3d),
    (3, 7, 5, (1e-5, 1.0), W.coeff_sines3d),
    (2, 63, 21, (1e-4,), None),               # m = 3969: several 1024-point LDS tiles and a ragged one
    (3, 15, 11, (1e-3,), W.coeff_sines3d),    # m = 3375, variable coefficient across tiles
]


@pytest.mark.parametrize("dim,nx,nt,gammas,coeff", KKT_CASES)
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("jchunk", [16, 3, -4, -16])
def test_kkt_apply(dim, nx, nt, gammas, coeff, transpose, jchunk):
    """Both matvec kernels (one thread per point marching jchunk levels; LDS
    tiles marching -jchunk levels), chunks that do not divide n included."""
    print(f"kkt_apply dim={dim} nx={nx} nt={nt} B={len(gammas)} var={coeff is not None} T={transpose} "
          f"jchunk={jchunk}", flush=True)
    spatial = "dst" if coeff is None else "mg"
    s = Solver(dim, nx, nt, list(gammas), coeff=coeff, spatial=spatial, kkt_jchunk=jchunk, device=DEV)
    assert s.kernels["kkt_jchunk"] == jchunk
    x = W.random_vector(dim, nx, nt, seed=1, batch=len(gammas))
    y = s.kkt_apply(to_dev(x), transpose=transpose).cpu().numpy()
    for b, pb in enumerate(problems(dim, nx, nt, gammas, coeff=coeff)):
        yo = D.kkt_apply(pb, x[b].ravel(), transpose=transpose)
        assert rel(y[b], yo) < 1e-14


def test_rhs_unpack_cotangent_datagrad():
    dim, nx, nt, gammas = 2, 15, 10, (1e-6, 1e-1)
    s = Solver(dim, nx, nt, list(gammas), device=DEV)
    fields = [W.random_fields(dim, nx, nt, seed=10 + b) for b in range(len(gammas))]
    g = np.stack([f[0] for f in fields])
    f = np.stack([f[1] for f in fields])
    y0 = np.stack([f[2] for f in fields])
    b = s.rhs(to_dev(g), to_dev(f), to_dev(y0)).cpu().numpy()
    lam = W.random_vector(dim, nx, nt, seed=3, batch=len(gammas))
    dg, df, dy0 = [t.cpu().numpy() for t in s.data_grad(to_dev(lam))]
    yb, pbar = np.random.default_rng(4).standard_normal((2, len(gammas), nt - 1, nx * nx))
    r = s.pack_cotangent(to_dev(yb), to_dev(pbar)).cpu().numpy()
    yy, pp = [t.cpu().numpy() for t in s.unpack(to_dev(lam))]
    for k, pb in enumerate(problems(dim, nx, nt, gammas)):
        assert rel(b[k], D.rhs_scaled(pb, g[k], f[k], y0[k])) < 1e-15
        og, of, oy0 = ADJ.data_gradients(pb, lam[k].ravel())
        assert rel(dg[k], og) < 1e-15 and rel(df[k], of) < 1e-15 and rel(dy0[k], oy0) < 1e-15
        assert rel(r[k], ADJ.loss_to_x_grad(pb, yb[k], pbar[k])) < 1e-15
        uy, up = D.unpack_solution(pb, lam[k].ravel())
        assert rel(yy[k], uy) < 1e-15 and rel(pp[k], up) < 1e-15


PRECOND_CASES = [
    # dim, nx, nt, gammas, eps
    (2, 15, 16, (1e-4,), None),          # n = 15 = 3 * 5
    (2, 31, 32, (1e-2, 1e-10), None),    # n = 31 prime, batch of two
    (2, 7, 9, (1.0,), 0.5),              # n = 8 = 4 * 2 (even n: self-paired Nyquist)
    (2, 15, 2, (1e-3,), None),           # n = 1
    (2, 15, 3, (1e-3,), None),           # n = 2
    (2, 63, 18, (1e-6,), 1.0 / 36),      # n = 17 prime, eps = tau/2
    (3, 7, 8, (1e-4,), None),            # 3-D sine transforms
    (2, 3, 13, (1e-4,), None),           # smallest sine length
    (2, 7, 20, (1e-4,), None),           # n = 19: chirp-z (Bluestein) time transform
    (2, 3, 128, (1e-6, 1e-2), None),     # n = 127: chirp-z, M = 256
    (2, 3, 512, (1e-6,), None),          # n = 511 = 7 * 73: chirp-z, M = 1024
    (2, 7, 256, (1e-2,), None),          # n = 255 = 3 * 5 * 17
    (2, 7, 65, (1e-3,), None),           # n = 64 = 8 * 8
    (2, 15, 12, (1e-3,), None),          # n = 11 (odd radix 11)
    (2, 7, 92, (1e-4,), None),           # n = 91 = 7 * 13
]


@pytest.mark.parametrize("dim,nx,nt,gammas,eps", PRECOND_CASES)
def test_precond_apply_fp64(dim, nx, nt, gammas, eps):
    print(f"precond fp64 dim={dim} nx={nx} nt={nt} B={len(gammas)}", flush=True)
    s = Solver(dim, nx, nt, list(gammas), eps=eps, device=DEV)
    v = W.random_vector(dim, nx, nt, seed=7, batch=len(gammas))
    w = s.precond_apply(to_dev(v)).cpu().numpy()
    wo = np.stack([P.EpsCirculantRBD(pb).apply(v[b].ravel()) for b, pb in enumerate(problems(dim, nx, nt, gammas, eps=eps))])
    for b in range(len(gammas)):
        assert rel(w[b], wo[b]) < 1e-11, rel(w[b], wo[b])
    check(w, wo, 1e-11, len(gammas), nt - 1, nx ** dim, label="fp64 apply")


@pytest.mark.parametrize("dim,nx,nt,gammas,eps", PRECOND_CASES[:3] + PRECOND_CASES[8:11])
def test_precond_apply_mixed(dim, nx, nt, gammas, eps):
    s = Solver(dim, nx, nt, list(gammas), eps=eps, precision="mixed", side="flexible", device=DEV)
    v = W.random_vector(dim, nx, nt, seed=8, batch=len(gammas))
    w = s.precond_apply(to_dev(v)).cpu().numpy()
    wo = np.stack([P.EpsCirculantRBD(pb).apply(v[b].ravel()) for b, pb in enumerate(problems(dim, nx, nt, gammas, eps=eps))])
    for b in range(len(gammas)):
        err = rel(w[b], wo[b])
        print(f"mixed precond rel err {err:.2e}")
        assert err < 1e-5
    check(w, wo, 1e-5, len(gammas), nt - 1, nx ** dim, label="mixed apply")


KERNEL_CASES = [
    # dim, nx, nt, gammas: time lengths with every radix mix the planner makes
    (2, 15, 16, (1e-4, 1e-8)),   # n = 15 = 3 * 5, two members
    (2, 7, 256, (1e-2,)),        # n = 255 = 3 * 5 * 17
    (2, 7, 65, (1e-3,)),         # n = 64 = 8 * 8
    (2, 15, 12, (1e-3,)),        # n = 11
    (2, 7, 9, (1.0,)),           # n = 8
    (2, 15, 2, (1e-3,)),         # n = 1
    (3, 7, 8, (1e-4,)),          # 3-D
    (2, 31, 513, (1e-6,)),       # n = 512: FP64 in-place blocks of 8 at most
    (2, 7, 15, (1e-3,)),         # n = 14 = 2 * 7
    (2, 3, 92, (1e-5,)),         # n = 91 = 7 * 13
]


@pytest.mark.parametrize("dim,nx,nt,gammas", KERNEL_CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_precond_kernel_choices(dim, nx, nt, gammas, precision):
    """Every time-pass kernel choice (two LDS buffers or in place, with 4, 8
    or 16 points per block) with both sine-transform kernels matches the oracle,
    and the choices agree with each other to rounding.  They do the same
    operations, but contraction into FMAs may differ between kernels; in FP32
    that rounding (~6e-8 per operation) is amplified by up to 1/eps = 16 in the
    last time levels by D_eps^{-1}, hence 1e-5 there."""
    print(f"kernel choices {precision} dim={dim} nx={nx} nt={nt} B={len(gammas)}", flush=True)
    side = "flexible" if precision == "mixed" else "right"
    v = W.random_vector(dim, nx, nt, seed=17, batch=len(gammas))
    wos = [P.EpsCirculantRBD(pb).apply(v[b].ravel()) for b, pb in enumerate(problems(dim, nx, nt, gammas))]
    tol = 1e-5 if precision == "mixed" else 1e-11
    for dk in (1, 2, 3, 4, 5):
        ref = None
        for tc in (-1, -16, -8, -4, 4, 8, 16):
            s = Solver(dim, nx, nt, list(gammas), precision=precision, side=side, time_cols=tc, dst_kernel=dk,
                       device=DEV)
            assert s.kernels["dst_kernel"] == dk
            eff = s.kernels["time_cols"]
            assert eff in (-16, -8, -4, 4, 8, 16)
            if (eff < 0) == (tc < 0) and tc != -1:
                assert abs(eff) <= abs(tc)
            w = s.precond_apply(to_dev(v)).cpu().numpy()
            for b in range(len(gammas)):
                assert rel(w[b], wos[b]) < tol, (dk, tc, eff, b, rel(w[b], wos[b]))
            check(w, np.stack(wos), tol, len(gammas), nt - 1, nx ** dim, label=f"dst {dk} time {eff}")
            if ref is None:
                ref = w
            else:
                assert rel(w, ref) < (1e-5 if precision == "mixed" else 1e-14), (dk, tc, eff)


HALF_DST_CASES = [
    # dim, nx, nt, gammas: strided sine transforms through a half-length FFT
    # (nx + 1 points, (nx + 1)/8 threads per line: 8, 16, 32 and 64, the
    # prefix sum of the odd outputs spanning up to a whole wavefront)
    (2, 63, 6, (1e-4, 1e-8)),
    (2, 127, 5, (1e-3,)),
    (2, 255, 4, (1e-6,)),
    (2, 511, 3, (1e-5,)),
    (3, 31, 5, (1e-3,)),       # both strided axes of 3-D
]


@pytest.mark.parametrize("dim,nx,nt,gammas", HALF_DST_CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_half_length_dst(dim, nx, nt, gammas, precision):
    """dst_kernel = 4 (strided lines through a half-length FFT and a prefix
    sum) and 5 (the same for the contiguous lines too) against the oracle
    and against the full-length register kernel (different operations:
    agreement to rounding of the transforms)."""
    print(f"half-length dst {precision} dim={dim} nx={nx} nt={nt} B={len(gammas)}", flush=True)
    side = "flexible" if precision == "mixed" else "right"
    v = W.random_vector(dim, nx, nt, seed=29, batch=len(gammas))
    ws = {}
    for dk in (1, 4, 5):
        s = Solver(dim, nx, nt, list(gammas), precision=precision, side=side, dst_kernel=dk, device=DEV)
        assert s.kernels["dst_kernel"] == dk
        ws[dk] = s.precond_apply(to_dev(v)).cpu().numpy()
    tol = 1e-5 if precision == "mixed" else 1e-11
    wo = np.stack([P.EpsCirculantRBD(pb).apply(v[b].ravel()) for b, pb in enumerate(problems(dim, nx, nt, gammas))])
    for dk in (4, 5):
        for b in range(len(gammas)):
            assert rel(ws[dk][b], wo[b]) < tol, (dk, b, rel(ws[dk][b], wo[b]))
        check(ws[dk], wo, tol, len(gammas), nt - 1, nx ** dim, label=f"half-length dst {dk}")
        assert rel(ws[dk], ws[1]) < (1e-5 if precision == "mixed" else 1e-12), (dk, rel(ws[dk], ws[1]))


CHIRP_CASES = [
    # dim, nx, nt, gammas: lengths with a prime factor above 17 (chirp-z)
    (2, 7, 20, (1e-4, 1e-8)),    # n = 19, M = 64, two members
    (2, 15, 128, (1e-6,)),       # n = 127, M = 256 (the 127-point workloads)
    (2, 3, 512, (1e-6,)),        # n = 511 = 7 * 73, M = 1024
    (2, 3, 1024, (1e-4,)),       # n = 1023 = 3 * 11 * 31, M = 2048
    (2, 3, 2048, (1e-4,)),       # n = 2047 = 23 * 89, M = 4096: FP64 tables stay in global memory
    (2, 3, 1153, (1e-4,)),       # n = 1152 = 2^7 3^2: smooth, but no radix tile fits LDS (M = 4096)
    (2, 3, 2049, (1e-4,)),       # n = 2048: chirp-z in FP64 (M = 4096), radix kernels in FP32
]


@pytest.mark.parametrize("nt,precision", [(1153, "fp64"), (1153, "mixed"), (2049, "fp64"), (1537, "fp64")])
def test_long_smooth_lengths_use_chirp(nt, precision):
    """Smooth lengths whose radix tiles do not fit LDS run the chirp-z kernels
    (M = 4096 allows at most 2 points per block) instead of being refused."""
    side = "flexible" if precision == "mixed" else "right"
    s = Solver(2, 3, nt, [1e-4], precision=precision, side=side, device=DEV)
    assert s.kernels["time_cols"] in (1, 2), s.kernels


@pytest.mark.parametrize("dim,nx,nt,gammas", CHIRP_CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_chirp_kernel_choices(dim, nx, nt, gammas, precision):
    """Every chirp-z kernel -- the three-stage convolution (+-32: 256 or 512
    threads) and the two-FFT kernels (points per block with 256 or 512
    threads) -- matches the oracle, and the shapes agree with each other to rounding (same
    operations per element; FMA contraction may differ between instances, and
    the two length-M FFTs of the convolution add about log2 M roundings of
    the largest spectral values, hence 1e-13 in FP64).  In FP32 the two FFTs
    give errors of about u log2 M (u = 6e-8), which D_eps^{-1} amplifies by up
    to 1/eps = sqrt(n) in the last time levels: the bar is twice that product,
    at least 1e-5."""
    print(f"chirp-z choices {precision} dim={dim} nx={nx} nt={nt} B={len(gammas)}", flush=True)
    side = "flexible" if precision == "mixed" else "right"
    v = W.random_vector(dim, nx, nt, seed=23, batch=len(gammas))
    wos = [P.EpsCirculantRBD(pb).apply(v[b].ravel()) for b, pb in enumerate(problems(dim, nx, nt, gammas))]
    n = nt - 1
    M = 1 << (2 * n - 2).bit_length()
    tol32 = max(1e-5, 2 * 6e-8 * np.log2(M) * np.sqrt(n))
    tol = tol32 if precision == "mixed" else 1e-11
    ref, seen = None, set()
    for tc in (0, 32, -32, 16, 8, 4, -16, -8, -4):
        s = Solver(dim, nx, nt, list(gammas), precision=precision, side=side, time_cols=tc, device=DEV)
        eff = s.kernels["time_cols"]
        assert eff in (64, -64, 32, -32, 16, 8, 4, 2, 1, -16, -8, -4), eff
        if tc != 0 and (eff < 0) == (tc < 0):
            assert abs(eff) <= abs(tc)
        if eff in seen:
            continue
        seen.add(eff)
        w = s.precond_apply(to_dev(v)).cpu().numpy()
        for b in range(len(gammas)):
            assert rel(w[b], wos[b]) < tol, (tc, eff, b, rel(w[b], wos[b]))
        check(w, np.stack(wos), tol, len(gammas), nt - 1, nx ** dim, label=f"chirp-z {eff}")
        if ref is None:
            ref = w
        else:
            assert rel(w, ref) < (tol32 if precision == "mixed" else 1e-13), (tc, eff, rel(w, ref))
    print(f"  shapes run: {sorted(seen)}", flush=True)


PRIME_FACTOR_CASES = [
    # dim, nx, nt, gammas: n = 511 = 7 x 73 (8-point tiles, and 16-point ones
    # in FP64 or 28 / 32-point ones with 1024 threads in FP32)
    (2, 3, 512, (1e-6,)),          # m = 9: one full 8-point tile and a ragged one; one ragged wide tile
    (2, 7, 512, (1e-4, 1e-8)),     # m = 49: six full 8-point tiles and a ragged one, two members; ragged wide tiles
    (3, 3, 512, (1e-3,)),          # 3-D, m = 27
    # n = 127 prime (16- and 32-point tiles, a 126-point Rader convolution)
    (2, 7, 128, (1e-4, 1e-8)),     # m = 49, ragged, two members
    (3, 3, 128, (1e-3,)),          # 3-D, m = 27
    # n = 255 = 15 x 17 (15- and 30-point tiles, a 16-point Rader convolution)
    (2, 15, 256, (1e-6,)),         # m = 225: 15 full 15-point tiles, 30-point tiles ragged
    (2, 7, 256, (1e-4, 1e-8)),     # m = 49, ragged, two members
]


@pytest.mark.parametrize("dim,nx,nt,gammas", PRIME_FACTOR_CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_prime_factor_time_kernels(dim, nx, nt, gammas, precision):
    """time_cols = +-64: the time passes by the Good-Thomas split with Rader
    transforms (n = 511 = 7 x 73: 73 points, n = 255 = 15 x 17: 17 points,
    n = 127: 127 points; the cyclic convolution in three LDS stages) against
    the oracle, and against the chirp-z kernels (n = 511) or the automatic
    kernels (different operations: agreement to rounding; in FP32 the bar of
    the chirp-z kernel-choice test, 2 u log2(M) sqrt(n))."""
    print(f"prime-factor time kernels {precision} dim={dim} nx={nx} nt={nt} B={len(gammas)}", flush=True)
    side = "flexible" if precision == "mixed" else "right"
    v = W.random_vector(dim, nx, nt, seed=31, batch=len(gammas))
    wos = np.stack([P.EpsCirculantRBD(pb).apply(v[b].ravel()) for b, pb in enumerate(problems(dim, nx, nt, gammas))])
    n = nt - 1
    M = 1 << (2 * n - 2).bit_length()
    tol32 = max(1e-5, 2 * 6e-8 * np.log2(M) * np.sqrt(n))
    tol = tol32 if precision == "mixed" else 1e-11
    ref_tc = 32 if n == 511 else 0
    ws = {}
    for tc in (64, -64, ref_tc):
        s = Solver(dim, nx, nt, list(gammas), precision=precision, side=side, time_cols=tc, device=DEV)
        if tc != 0:
            assert s.kernels["time_cols"] == tc, s.kernels
        ws[tc] = s.precond_apply(to_dev(v)).cpu().numpy()
    for tc in (64, -64):
        for b in range(len(gammas)):
            assert rel(ws[tc][b], wos[b]) < tol, (tc, b, rel(ws[tc][b], wos[b]))
        check(ws[tc], wos, tol, len(gammas), n, nx ** dim, label=f"prime-factor {tc}")
        assert rel(ws[tc], ws[ref_tc]) < (tol32 if precision == "mixed" else 1e-13), (tc, rel(ws[tc], ws[ref_tc]))
    # the two tile widths run the same operations per element
    assert rel(ws[64], ws[-64]) < (1e-6 if precision == "mixed" else 1e-15), rel(ws[64], ws[-64])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_prime_factor_solve_matches_chirp(precision):
    """A whole solve with the prime-factor time kernels (scaled inputs of the
    Krylov basis, accumulated outputs) takes the iterations of the chirp-z
    solve and reaches the same solution."""
    side = "flexible" if precision == "mixed" else "right"
    gammas = [1e-4, 1e-6]
    dim, nx, nt = 2, 15, 512
    rng = np.random.default_rng(37)
    out = {}
    for tc in (-64, 32):
        s = Solver(dim, nx, nt, gammas, precision=precision, side=side, time_cols=tc, device=DEV)
        assert s.kernels["time_cols"] == tc
        b = to_dev(rng.standard_normal(tuple(s.vec_shape))) if tc == -64 else b
        x, infos, _ = s.solve(b)
        out[tc] = (x.cpu().numpy(), [i.iters for i in infos])
    print(f"prime-factor solve {precision}: iterations {out[-64][1]} vs chirp-z {out[32][1]}", flush=True)
    assert out[-64][1] == out[32][1]
    assert rel(out[-64][0], out[32][0]) < 1e-9


def test_tuned_solve_matches_default():
    """tune = 1 picks kernels by timing; the solve gives the same iterate."""
    dim, nx, nt, gammas = 2, 31, 64, (1e-2, 1e-6)
    fields = [W.random_fields(dim, nx, nt, seed=40 + b) for b in range(len(gammas))]
    g, f, y0 = (to_dev(np.stack([fl[i] for fl in fields])) for i in range(3))
    out = {}
    for tune in (False, True):
        s = Solver(dim, nx, nt, list(gammas), tune=tune, device=DEV)
        print(f"tune={tune} kernels {s.kernels}", flush=True)
        if tune:
            assert s.kernels["tuned_ms"] > 0
        x, infos, _ = s.solve(s.rhs(g, f, y0))
        out[tune] = (x.cpu().numpy(), [i.iters for i in infos])
    assert out[True][1] == out[False][1]
    assert rel(out[True][0], out[False][0]) < 1e-12


MG_CASES = [
    # dim, nx, nt, gammas, coefficient
    (2, 15, 16, (1e-4,), None),
    (2, 15, 12, (1e-3, 1e-8), W.coeff_sines3d),
    (3, 7, 9, (1e-5,), W.coeff_sines3d),
    (3, 15, 8, (1e-2,), W.coeff_sines3d),
    (2, 1, 5, (1e-3,), W.coeff_sines3d),      # single-point grid: the cycle is an exact solve
    (2, 31, 20, (1e-6,), W.coeff_example2),   # Example 2 coefficient, chirp-z time transform
    # shapes whose finest level runs the smoother, residual and prolongation
    # with eight slices per thread (at least 1024 blocks of 256 points x 8
    # slices); coarser levels fall back to one slice per thread
    (2, 127, 128, (1e-5,), W.coeff_sines3d),  # 64 point blocks x 16 slice groups
    (2, 127, 130, (1e-4,), W.coeff_example2), # 130 slices: the last group holds 2
    (3, 31, 72, (1e-5,), W.coeff_sines3d),    # 117 x 9 groups (72 slices)
    (3, 31, 38, (1e-3, 1e-7), W.coeff_sines3d),  # 76 slices: member boundary inside a group, tail of 4
]


def mg_wide_levels(dim, nx, nt, batch):
    """Levels that take the eight-slices-per-thread kernels (the launch rule
    of the multigrid cycle: ceil(m/256) * ceil(slices/8) >= 1024)."""
    slices = batch * 2 * ((nt - 1) // 2 + 1)
    out = []
    while True:
        out.append(((nx ** dim + 255) // 256) * ((slices + 7) // 8) >= 1024)
        if nx == 1:
            return out
        nx = (nx - 1) // 2


@pytest.mark.parametrize("dim,nx,nt,gammas,coeff", MG_CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_precond_apply_multigrid(dim, nx, nt, gammas, coeff, precision):
    wide = mg_wide_levels(dim, nx, nt, len(gammas))
    print(f"precond mg {precision} dim={dim} nx={nx} nt={nt} B={len(gammas)} eight-slice levels {wide}", flush=True)
    side = "flexible" if precision == "mixed" else "right"
    s = Solver(dim, nx, nt, list(gammas), coeff=coeff, spatial="mg", precision=precision, side=side, device=DEV)
    v = W.random_vector(dim, nx, nt, seed=17, batch=len(gammas))
    w = s.precond_apply(to_dev(v)).cpu().numpy()
    wo = np.stack([P.EpsCirculantRBD(pb, spatial="mg", coeff=coeff).apply(v[b].ravel())
                   for b, pb in enumerate(problems(dim, nx, nt, gammas, coeff=coeff))])
    check(w, wo, 1e-11 if precision == "fp64" else 1e-5, len(gammas), nt - 1, nx ** dim, label="mg apply")


LEX_CASES = [
    # dim, nx, nt, gammas, coefficient: the lexicographic smoothers
    (2, 15, 12, (1e-3, 1e-8), W.coeff_sines3d),
    (2, 31, 20, (1e-2,), W.coeff_example2),
    (3, 7, 9, (1e-5,), W.coeff_sines3d),
    (2, 1, 5, (1e-3,), W.coeff_sines3d),       # single point: the sweep is the exact solve
    (2, 127, 130, (1e-4,), W.coeff_example2),  # the residual kernel with eight slices per thread
    (3, 31, 38, (1e-3, 1e-7), W.coeff_sines3d),
]


@pytest.mark.parametrize("dim,nx,nt,gammas,coeff", LEX_CASES)
@pytest.mark.parametrize("smoother", ["lex", "sym"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_precond_apply_multigrid_lexicographic(dim, nx, nt, gammas, coeff, smoother, precision):
    """mg_smoother = 1 / 2: the V-cycle with a Gauss-Seidel sweep in the
    natural order (then the reverse order) against the oracle's cycle with
    the same smoother."""
    print(f"precond mg {smoother} {precision} dim={dim} nx={nx} nt={nt} B={len(gammas)}", flush=True)
    side = "flexible" if precision == "mixed" else "right"
    s = Solver(dim, nx, nt, list(gammas), coeff=coeff, spatial="mg", precision=precision, side=side,
               mg_smoother=smoother, device=DEV)
    v = W.random_vector(dim, nx, nt, seed=19, batch=len(gammas))
    w = s.precond_apply(to_dev(v)).cpu().numpy()
    wo = np.stack([P.EpsCirculantRBD(pb, spatial="mg", coeff=coeff, smoother=smoother).apply(v[b].ravel())
                   for b, pb in enumerate(problems(dim, nx, nt, gammas, coeff=coeff))])
    check(w, wo, 1e-11 if precision == "fp64" else 1e-5, len(gammas), nt - 1, nx ** dim, label=f"mg {smoother}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_multigrid_flexible_solve(precision):
    # 3-D sparse direct solves grow quickly on the host: keep the oracle side small
    dim, nx, nt, gamma = 3, 7, 16, 1e-5
    g, f, y0 = W.random_fields(dim, nx, nt, seed=71)
    s = Solver(dim, nx, nt, gamma, coeff=W.coeff_sines3d, spatial="mg", precision=precision, side="flexible",
               device=DEV)
    x, infos, _ = s.solve(s.rhs(to_dev(g[None]), to_dev(f[None]), to_dev(y0[None])))
    assert infos[0].converged and infos[0].relres_true <= 1.05e-8
    pb = D.make_problem(dim, nx, nt, gamma, coeff=W.coeff_sines3d)
    xo = spla.spsolve(D.kkt_scaled(pb).tocsc(), D.rhs_scaled(pb, g, f, y0))
    assert rel(x.cpu().numpy(), xo) < 1e-6


def test_precond_in_place():
    s = Solver(2, 15, 16, 1e-4, device=DEV)
    v = to_dev(W.random_vector(2, 15, 16, seed=9))
    w = s.precond_apply(v)
    v2 = v.clone()
    s.precond_apply(v2, out=v2)
    assert torch.equal(w, v2)


@pytest.mark.parametrize("side", ["right", "left", "flexible"])
def test_fixed_k_iterates_match_oracle(side):
    """Same side, same k Arnoldi steps, x0 = 0: the iterates agree (CGS on the
    GPU, MGS in the oracle: equal in exact arithmetic)."""
    dim, nx, nt, gamma = 2, 15, 16, 1e-4
    g, f, y0 = W.random_fields(dim, nx, nt, seed=21)
    pb = D.make_problem(dim, nx, nt, gamma)
    A = D.kkt_scaled(pb)
    bo = D.rhs_scaled(pb, g, f, y0)
    pc = P.EpsCirculantRBD(pb)
    for k in (1, 3, 6):
        s = Solver(dim, nx, nt, gamma, side=side, maxit=k, rtol=1e-30, device=DEV)
        b = s.rhs(to_dev(g[None]), to_dev(f[None]), to_dev(y0[None]))
        x, infos, hist = s.solve(b, history=True)
        res = KR.gmres(lambda v: A @ v, bo, pc.apply, side=side, fixed_iters=k)
        assert infos[0].iters == k
        assert rel(x.cpu().numpy(), res.x) < 1e-10
        np.testing.assert_allclose(hist[0, : k + 1], res.history[: k + 1], rtol=1e-8)


@pytest.mark.parametrize("side", ["right", "left", "flexible"])
def test_long_iterates_across_restart_match_oracle(side):
    """k = 8, 20, 30 and 35 Arnoldi steps of GMRES(30) (35 crosses the
    restart) on a slowly converging problem (eps near 1 and a short horizon,
    so the preconditioned spectrum spreads and the residual is still about
    1e-6 at step 35): every basis size up to 31 and the restarted cycle are
    compared with the oracle's iterate and residual history."""
    dim, nx, nt, gamma, eps, T = 2, 15, 24, 1e-3, 0.99, 0.005
    g, f, y0 = W.random_fields(dim, nx, nt, seed=21)
    pb = D.make_problem(dim, nx, nt, gamma, eps=eps, T=T)
    A = D.kkt_scaled(pb)
    bo = D.rhs_scaled(pb, g, f, y0)
    pc = P.EpsCirculantRBD(pb)
    for k in (8, 20, 30, 35):
        s = Solver(dim, nx, nt, gamma, T=T, eps=eps, side=side, restart=30, maxit=k, rtol=1e-30, device=DEV)
        b = s.rhs(to_dev(g[None]), to_dev(f[None]), to_dev(y0[None]))
        x, infos, hist = s.solve(b, history=True)
        res = KR.gmres(lambda v: A @ v, bo, pc.apply, side=side, restart=30, maxit=k, rtol=1e-30)
        assert infos[0].iters == k == res.iters
        err = rel(x.cpu().numpy(), res.x)
        hd = np.abs(hist[0, : k + 1] - np.asarray(res.history[: k + 1]))
        print(f"  {side} k={k}: x rel err {err:.2e}, residual {res.history[k]:.2e}, "
              f"history max rel diff {np.max(hd / np.asarray(res.history[: k + 1])):.2e}", flush=True)
        assert err < 1e-10
        # the estimates are |g_{k+1}| / beta0 with g rotated from beta0 e_1, so
        # their rounding is absolute (a few hundred ulps of 1), not relative
        np.testing.assert_allclose(hist[0, : k + 1], res.history[: k + 1], rtol=1e-8, atol=1e-13)


MIXED_SOLVE_CASES = [
    # dim, nx, nt, gamma: FP32 preconditioner in FP64 flexible GMRES at 1e-8
    (2, 31, 32, 1e-2),
    (2, 31, 32, 1e-4),
    (2, 31, 32, 1e-6),
    (2, 31, 32, 1e-10),
    (2, 63, 64, 1e-6),
    (2, 15, 128, 1e-2),   # n = 127: chirp-z time transform in FP32
]


@pytest.mark.parametrize("dim,nx,nt,gamma", MIXED_SOLVE_CASES)
def test_mixed_solve_matches_fp64_oracle(dim, nx, nt, gamma):
    """The mixed path (complex-FP32 P_eps^{-1}; matvec, Arnoldi and residuals
    in FP64) stopped at the true relative residual 1e-8 against the oracle's
    all-FP64 flexible GMRES stopped at the same residual: relative error at
    most 1e-7.  The error against the exact solution x* = A^{-1} b is printed
    for each result."""
    g, f, y0 = W.random_fields(dim, nx, nt, seed=101)
    pb = D.make_problem(dim, nx, nt, gamma)
    A = D.kkt_scaled(pb)
    bo = D.rhs_scaled(pb, g, f, y0)
    res = KR.gmres(lambda v: A @ v, bo, P.EpsCirculantRBD(pb).apply, side="flexible", rtol=1e-8, restart=30,
                   maxit=300)
    assert res.converged
    s = Solver(dim, nx, nt, gamma, precision="mixed", side="flexible", rtol=1e-8, device=DEV)
    x, infos, _ = s.solve(s.rhs(to_dev(g[None]), to_dev(f[None]), to_dev(y0[None])))
    assert infos[0].converged and infos[0].relres_true <= 1e-8 * 1.0001, infos[0]
    xg = x.cpu().numpy().ravel()
    e_orc = rel(xg, res.x)
    msg = (f"  mixed dim={dim} nx={nx} nt={nt} gamma={gamma:g}: iters gpu {infos[0].iters} oracle {res.iters}; "
           f"rel err vs FP64 oracle iterate {e_orc:.2e}")
    if A.shape[0] <= 100000:  # a sparse direct solve of the whole system stays quick
        xstar = spla.spsolve(A.tocsc(), bo)
        msg += f", vs x* {rel(xg, xstar):.2e} (oracle iterate vs x* {rel(res.x, xstar):.2e})"
    print(msg, flush=True)
    assert e_orc <= 1e-7


def test_resume_from_nonzero_initial_guess():
    """GMRES(5) stopped after 5 steps and called again from the returned x
    continues exactly as one 10-step call (the second call starts the second
    restart cycle from the same residual)."""
    dim, nx, nt, gamma = 2, 15, 24, 1e-3
    g, f, y0 = W.random_fields(dim, nx, nt, seed=21)
    kw = dict(T=0.005, eps=0.99, restart=5, rtol=1e-30, device=DEV)
    s10 = Solver(dim, nx, nt, gamma, maxit=10, **kw)
    b = s10.rhs(to_dev(g[None]), to_dev(f[None]), to_dev(y0[None]))
    x10, i10, _ = s10.solve(b)
    s5 = Solver(dim, nx, nt, gamma, maxit=5, **kw)
    x5, i5, _ = s5.solve(b)
    xr, ir, _ = s5.solve(b, x0=x5)
    assert i10[0].iters == 10 and i5[0].iters == 5 and ir[0].iters == 5
    err = rel(xr.cpu().numpy(), x10.cpu().numpy())
    print(f"  resumed vs uninterrupted: {err:.2e}; true residuals {ir[0].relres_true:.3e} {i10[0].relres_true:.3e}")
    assert err < 1e-12
    assert abs(ir[0].relres_true - i10[0].relres_true) <= 1e-8 * i10[0].relres_true + 1e-15
    # and the oracle's restarted GMRES(5) from the same initial guess
    pb = D.make_problem(dim, nx, nt, gamma, eps=0.99, T=0.005)
    A = D.kkt_scaled(pb)
    res = KR.gmres(lambda v: A @ v, b.cpu().numpy().ravel(), P.EpsCirculantRBD(pb).apply, side="right",
                   x0=x5.cpu().numpy().ravel(), restart=5, maxit=5, rtol=1e-30)
    assert rel(xr.cpu().numpy(), res.x) < 1e-10


@pytest.mark.parametrize("side", ["right", "flexible"])
def test_solve_converges_to_direct_solution(side):
    dim, nx, nt, gammas = 2, 31, 32, (1e-2, 1e-6, 1e-10)
    fields = [W.fields(W.WORKLOADS["2d-nx31-nt32"], member=b) for b in range(3)]
    s = Solver(dim, nx, nt, list(gammas), side=side, device=DEV)
    g = np.stack([fl[0] for fl in fields])
    f = np.stack([fl[1] for fl in fields])
    y0 = np.stack([fl[2] for fl in fields])
    b = s.rhs(to_dev(g), to_dev(f), to_dev(y0))
    x, infos, _ = s.solve(b)
    xs = x.cpu().numpy()
    for k, pb in enumerate(problems(dim, nx, nt, gammas)):
        assert infos[k].converged and infos[k].relres_true <= 1e-8 * 1.05, infos[k]
        xo = spla.spsolve(D.kkt_scaled(pb).tocsc(), D.rhs_scaled(pb, g[k], f[k], y0[k]))
        assert rel(xs[k], xo) < 1e-6


@pytest.mark.parametrize("reorth_tol", [0.0, -1.0])
def test_reorthogonalisation_switch(reorth_tol):
    """Always running the second Gram-Schmidt pass (0) or never (-1) gives the
    same iterates as the measured default to rounding."""
    dim, nx, nt, gamma = 2, 15, 16, 1e-3
    g, f, y0 = W.random_fields(dim, nx, nt, seed=33)
    xs = []
    its = []
    for tol in (1e-8, reorth_tol):
        s = Solver(dim, nx, nt, gamma, reorth_tol=tol, device=DEV)
        x, infos, _ = s.solve(s.rhs(to_dev(g[None]), to_dev(f[None]), to_dev(y0[None])))
        assert infos[0].converged
        xs.append(x.cpu().numpy())
        its.append(infos[0].iters)
    assert its[0] == its[1]
    assert rel(xs[1], xs[0]) < 1e-11


@pytest.mark.parametrize("nt", [16, 32])
def test_batched_member_equals_single_solve(nt):
    """Each member of a batched solve (members converge at different steps,
    so later steps run with member masks) matches its own single solve;
    nt = 32 runs the chirp-z time kernels (n = 31)."""
    dim, nx, gammas = 2, 15, (1e-2, 1e-7, 1e-4)
    fields = [W.random_fields(dim, nx, nt, seed=40 + b) for b in range(3)]
    g = np.stack([fl[0] for fl in fields])
    f = np.stack([fl[1] for fl in fields])
    y0 = np.stack([fl[2] for fl in fields])
    sb = Solver(dim, nx, nt, list(gammas), device=DEV)
    xb, ib, _ = sb.solve(sb.rhs(to_dev(g), to_dev(f), to_dev(y0)))
    for k, gm in enumerate(gammas):
        s1 = Solver(dim, nx, nt, gm, device=DEV)
        x1, i1, _ = s1.solve(s1.rhs(to_dev(g[k:k + 1]), to_dev(f[k:k + 1]), to_dev(y0[k:k + 1])))
        assert i1[0].iters == ib[k].iters
        assert rel(xb[k].cpu().numpy(), x1[0].cpu().numpy()) < 1e-13


@pytest.mark.parametrize("chunk", [1, 3, 4])
def test_graph_solve_matches_eager(chunk):
    """Arnoldi chunks replayed as captured HIP graphs give the eager solve's
    iterates; the graphs are replayed across several solves with eager work
    in between."""
    dim, nx, nt, gammas = 2, 15, 16, (1e-2, 1e-7, 1e-4)
    fields = [W.random_fields(dim, nx, nt, seed=80 + b) for b in range(3)]
    g = np.stack([fl[0] for fl in fields])
    f = np.stack([fl[1] for fl in fields])
    y0 = np.stack([fl[2] for fl in fields])
    se = Solver(dim, nx, nt, list(gammas), device=DEV)
    xe, ie, he = se.solve(se.rhs(to_dev(g), to_dev(f), to_dev(y0)), history=True)
    sg = Solver(dim, nx, nt, list(gammas), graph=True, graph_chunk=chunk, device=DEV)
    b = sg.rhs(to_dev(g), to_dev(f), to_dev(y0))
    for rep in range(3):
        xg, ig, hg = sg.solve(b, history=True)
        for k in range(3):
            assert ig[k].converged and ig[k].iters == ie[k].iters
            assert rel(xg[k].cpu().numpy(), xe[k].cpu().numpy()) < 1e-14
        np.testing.assert_array_equal(np.nan_to_num(hg), np.nan_to_num(he))
        sg.kkt_apply(b)  # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("spatial,precision", [("mg", "fp64"), ("mg", "mixed"), ("dst", "mixed")])
def test_graph_flexible_solve_matches_eager(spatial, precision):
    """Graph mode on the flexible paths: the multigrid V-cycle (FP64 and
    FP32) and the FP32 sine-transform preconditioner inside flexible GMRES,
    replayed across solves with eager work in between, give the eager
    iterates (no reductions by atomics, so the same kernels give the same
    bits)."""
    if spatial == "mg":
        dim, nx, nt, gammas, coeff = 3, 7, 12, (1e-3, 1e-6), W.coeff_sines3d
    else:
        dim, nx, nt, gammas, coeff = 2, 15, 16, (1e-2, 1e-7), None
    print(f"graph flexible {spatial} {precision} dim={dim} nx={nx} nt={nt}", flush=True)
    fields = [W.random_fields(dim, nx, nt, seed=60 + b) for b in range(len(gammas))]
    g = np.stack([fl[0] for fl in fields])
    f = np.stack([fl[1] for fl in fields])
    y0 = np.stack([fl[2] for fl in fields])
    kw = dict(coeff=coeff, spatial=spatial, precision=precision, side="flexible", device=DEV)
    se = Solver(dim, nx, nt, list(gammas), **kw)
    xe, ie, he = se.solve(se.rhs(to_dev(g), to_dev(f), to_dev(y0)), history=True)
    assert all(i.converged for i in ie)
    sg = Solver(dim, nx, nt, list(gammas), graph=True, graph_chunk=3, **kw)
    b = sg.rhs(to_dev(g), to_dev(f), to_dev(y0))
    for rep in range(3):
        xg, ig, hg = sg.solve(b, history=True)
        for k in range(len(gammas)):
            assert ig[k].converged and ig[k].iters == ie[k].iters, (rep, k, ig[k].iters, ie[k].iters)
        assert rel(xg.cpu().numpy(), xe.cpu().numpy()) < 1e-14, rep
        np.testing.assert_array_equal(np.nan_to_num(hg), np.nan_to_num(he))
        sg.kkt_apply(b)  # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("dim,nx,nt", [(2, 1, 4), (2, 3, 5), (3, 3, 6), (2, 7, 33), (2, 15, 20)])
def test_tuned_solve_tiny_shapes(dim, nx, nt):
    """With tune = 1 every kernel candidate runs on tiny shapes (a one-point
    grid through multigrid, tiles mostly empty, a chirp-z length); the tuned
    solve converges to the untuned one."""
    gammas = (1e-3, 1e-7)
    fields = [W.random_fields(dim, nx, nt, seed=95 + b) for b in range(2)]
    g = np.stack([fl[0] for fl in fields])
    f = np.stack([fl[1] for fl in fields])
    y0 = np.stack([fl[2] for fl in fields])
    spatial = "dst" if nx >= 3 else "mg"  # sine transforms need nx + 1 >= 4
    xs = {}
    for tune in (False, True):
        s = Solver(dim, nx, nt, list(gammas), spatial=spatial, side="flexible" if spatial == "mg" else "right",
                   tune=tune, device=DEV)
        print(f"tiny dim={dim} nx={nx} nt={nt} tune={tune} kernels {s.kernels}", flush=True)
        x, infos, _ = s.solve(s.rhs(to_dev(g), to_dev(f), to_dev(y0)))
        assert all(i.converged and i.relres_true <= 1e-8 * 1.001 for i in infos), infos
        xs[tune] = x.cpu().numpy()
    assert rel(xs[True], xs[False]) < 1e-6


def test_side_stream_solve_starts_from_zero():
    """A solver on its own stream (as graph mode requires) orders its work
    after the caller's stream: x0 = 0 is zero-filled on the caller's stream,
    so without that order a solve could read recycled memory as its initial
    guess.  Before each solve a freed block full of ones is left in torch's
    caching allocator; every solve must still match the eager solve."""
    dim, nx, nt, gammas = 2, 15, 16, (1e-2, 1e-7, 1e-4)
    fields = [W.random_fields(dim, nx, nt, seed=85 + b) for b in range(3)]
    g = np.stack([fl[0] for fl in fields])
    f = np.stack([fl[1] for fl in fields])
    y0 = np.stack([fl[2] for fl in fields])
    se = Solver(dim, nx, nt, list(gammas), device=DEV)
    xe, ie, _ = se.solve(se.rhs(to_dev(g), to_dev(f), to_dev(y0)))
    side = torch.cuda.Stream(device=DEV)
    sg = Solver(dim, nx, nt, list(gammas), graph=True, graph_chunk=3, device=DEV, stream=side)
    b = sg.rhs(to_dev(g), to_dev(f), to_dev(y0))
    for rep in range(4):
        junk = torch.ones(sg.vec_shape, dtype=torch.float64, device=DEV)
        del junk  # the next vector of this size may reuse the block
        xg, ig, _ = sg.solve(b)
        for k in range(3):
            assert ig[k].converged and ig[k].iters == ie[k].iters, (rep, k, ig[k].iters, ie[k].iters)
        assert rel(xg.cpu().numpy(), xe.cpu().numpy()) < 1e-13, rep


def test_transpose_solve():
    dim, nx, nt, gamma = 2, 15, 16, 1e-3
    pb = D.make_problem(dim, nx, nt, gamma)
    r = W.random_vector(dim, nx, nt, seed=50)
    s = Solver(dim, nx, nt, gamma, rtol=1e-12, device=DEV)
    lam, infos, _ = s.solve(to_dev(r), transpose=True)
    assert infos[0].converged
    lo = ADJ.adjoint_solve(pb, r.ravel())
    assert rel(lam.cpu().numpy(), lo) < 1e-9


ROWS = [  # (gamma, nx, nt, iters) from Tables 1 and 3 (Example 1, eps = tau/2, left GMRES)
    (1e-10, 31, 32, 6), (1e-8, 31, 64, 8), (1e-6, 31, 32, 10), (1e-6, 31, 256, 17),
    (1e-4, 31, 32, 15), (1e-2, 31, 32, 16), (1.0, 31, 32, 10), (1e-6, 63, 64, 12),
]


@pytest.mark.parametrize("gamma,nx,nt,iters", ROWS)
def test_paper_iteration_counts_left(gamma, nx, nt, iters):
    tau = 1.0 / nt
    g, f, y0 = W.example_fields(1, 2, nx, nt)
    s = Solver(2, nx, nt, gamma, eps=min(0.5, tau / 2), side="left", device=DEV)
    x, infos, _ = s.solve(s.rhs(to_dev(g[None]), to_dev(f[None]), to_dev(y0[None])))
    assert infos[0].converged
    assert infos[0].iters == iters


def test_autograd_matches_oracle_and_envelope():
    dim, nx, nt, gamma = 2, 15, 12, 1e-3
    g, f, y0 = W.random_fields(dim, nx, nt, seed=60)
    s = Solver(dim, nx, nt, gamma, rtol=1e-12, device=DEV)
    tg = to_dev(g[None]).requires_grad_(True)
    tf = to_dev(f[None]).requires_grad_(True)
    ty0 = to_dev(y0[None]).requires_grad_(True)
    y, p = kkt_solve(s, tg, tf, ty0)
    # J* = tau/2 ||y - g||^2 + gamma tau/2 ||p/gamma||^2: its total derivative is
    # the envelope closed form -tau (y - g), -tau p, -p^1
    J = 0.5 * s.tau * ((y - tg) ** 2).sum() + 0.5 * gamma * s.tau * ((p / gamma) ** 2).sum()
    J.backward()
    pb = D.make_problem(dim, nx, nt, gamma)
    yo, po = D.unpack_solution(pb, spla.spsolve(D.kkt_scaled(pb).tocsc(), D.rhs_scaled(pb, g, f, y0)))
    eg, ef, ey0 = ADJ.envelope_gradients(pb, yo, po, g)
    assert rel(tg.grad.cpu().numpy()[0], eg) < 1e-8
    assert rel(tf.grad.cpu().numpy()[0], ef) < 1e-8
    assert rel(ty0.grad.cpu().numpy()[0], ey0) < 1e-8


@pytest.mark.parametrize("side", ["right", "flexible"])
def test_gs_update_pairs_matches_scalar(side):
    """The double2 Gram-Schmidt update and the one-element update give the
    same iterates up to rounding (the dot products sum pairs first)."""
    dim, nx, nt, gammas = 2, 15, 24, (1e-3, 1e-7)
    fields = [W.random_fields(dim, nx, nt, seed=90 + b) for b in range(len(gammas))]
    g, f, y0 = (to_dev(np.stack([fl[i] for fl in fields])) for i in range(3))
    out = {}
    for gs in (1, 2):
        s = Solver(dim, nx, nt, list(gammas), side=side, gs_update=gs, device=DEV)
        assert s.kernels["gs_update"] == gs
        x, infos, _ = s.solve(s.rhs(g, f, y0))
        out[gs] = (x.cpu().numpy(), [i.iters for i in infos])
    assert out[1][1] == out[2][1]
    assert rel(out[1][0], out[2][0]) < 1e-12
