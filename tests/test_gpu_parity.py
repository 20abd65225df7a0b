"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances: rel-L2 <= 1e-12 for double-precision plans and <= 1e-6 for
single-precision plans, with the max-norm error reported beside it.  A
single-precision plan reads the density rounded to float32, so it is compared
against the oracle run on that same rounded density (input rounding is not
solver error).
"""
import numpy as np
import pytest

import oracle
from conftest import gpu_available
from paper_2409_02294_amd import inputs

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_2409_02294_amd import solver as S


TOL = {"f64": 1e-12, "f32": 1e-6, "f64_plain": 1e-12, "f32_plain": 1e-6, "f32_split": 1e-6}


def _dtype(prec):
    return torch.float64 if prec.startswith("f64") else torch.float32


def gpu_solve(rho_np, prec, dx=None, G=1.0, self_coeff=2.38):
    n = rho_np.shape[0]
    s = S.Solver(n, dx if dx is not None else 1.0 / n, prec, G=G, self_coeff=self_coeff)
    rho = torch.from_numpy(np.ascontiguousarray(rho_np)).to(device="cuda", dtype=_dtype(prec))
    phi = s(rho)
    torch.cuda.synchronize()
    return phi.cpu().numpy().astype(np.float64), rho.cpu().numpy().astype(np.float64), s


def _report(tag, got, ref):
    l2, mx = oracle.rel_l2(got, ref), oracle.rel_max(got, ref)
    print(f"{tag}: relL2={l2:.3e} relMax={mx:.3e}", flush=True)
    return l2, mx


# ---------------------------------------------------------------------------
# Single passes of the pruned pipeline against numpy's FFT, one axis at a time
# ---------------------------------------------------------------------------

def _ghat_octant(n, dx, G=1.0):
    p = 2 * n
    g = oracle.green_hat(n, dx).real * (G * dx ** 3 / p ** 3)   # [kz][ky][kx]
    h = n + 1
    return np.ascontiguousarray(np.transpose(g[:h, :h, :h], (2, 1, 0)))  # [kx][ky][kz]


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
@pytest.mark.parametrize("n", [8, 24, 32, 40, 48, 72, 120, 144])
def test_passes_match_numpy(prec, n):
    rng = np.random.default_rng(n)
    p, h = 2 * n, n + 1
    dt = _dtype(prec)
    cdt = torch.complex128 if dt == torch.float64 else torch.complex64
    tol = 1e-13 if prec == "f64" else 2e-6
    plan = S.Solver(n, 1.0 / n, prec)
    st = torch.cuda.current_stream().cuda_stream

    def run(pass_id, x_np, out_shape, out_complex):
        x = torch.from_numpy(x_np).to("cuda")
        x = x.to(cdt if np.iscomplexobj(x_np) else dt).contiguous()
        out = torch.empty(out_shape, dtype=cdt if out_complex else dt, device="cuda")
        S.ps_debug_pass(plan.plan, pass_id, x.data_ptr(), out.data_ptr(), st)
        torch.cuda.synchronize()
        return x.cpu().numpy().astype(np.complex128 if np.iscomplexobj(x_np) else np.float64), out.cpu().numpy()

    def check(tag, got, ref):
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"pass {tag} n={n} {prec}: rel max err {err:.2e}", flush=True)
        assert err <= tol

    # pass 0: real FFT along x with zero padding to P
    rho = rng.uniform(-1, 1, (n, n, n))
    rho_in, t1 = run(0, rho, (h, n, n), True)
    ref = np.transpose(np.fft.rfft(rho_in, n=p, axis=2), (2, 0, 1))
    check("x_r2c", t1, ref)
    # pass 1: FFT along y with zero padding
    a = rng.standard_normal((h, n, n)) + 1j * rng.standard_normal((h, n, n))
    a_in, t2 = run(1, a, (h, p, n), True)
    ref = np.transpose(np.fft.fft(a_in, n=p, axis=2), (0, 2, 1))
    check("y_fwd", t2, ref)
    # pass 2: FFT along z (zero padded), product with the kernel octant, inverse,
    # crop; output T3[kx][z][ky]
    b = rng.standard_normal((h, p, n)) + 1j * rng.standard_normal((h, p, n))
    b_in, t3 = run(2, b, (h, n, p), True)
    go = _ghat_octant(n, 1.0 / n)
    fold = np.minimum(np.arange(p), p - np.arange(p))
    gfull = go[:, fold, :][:, :, fold]                      # [kx][ky][kz]
    ref = np.fft.ifft(np.fft.fft(b_in, n=p, axis=2) * gfull, axis=2)[:, :, :n] * p
    check("z_conv", t3, np.transpose(ref, (0, 2, 1)))
    # pass 3: inverse FFT along y, crop; in T3[kx][z][ky], out T4[z][y][kx] (row pitch hp)
    hp = (h + 15) // 16 * 16
    c = rng.standard_normal((h, n, p)) + 1j * rng.standard_normal((h, n, p))
    c_in, t4 = run(3, c, (n, n, hp), True)
    ref = np.transpose(np.fft.ifft(c_in, axis=2)[:, :, :n] * p, (1, 2, 0))
    check("y_inv", t4[:, :, :h], ref)
    # pass 4: inverse real FFT along x, crop; the row padding beyond kx = n is ignored
    d = rng.standard_normal((n, n, hp)) + 1j * rng.standard_normal((n, n, hp))
    d[:, :, h:] = 1e30
    d_in, out = run(4, d, (n, n, n), False)
    ref = np.fft.irfft(d_in[:, :, :h], n=p, axis=2)[:, :, :n] * p
    check("x_c2r", out, ref)


# ---------------------------------------------------------------------------
# Whole solves against the oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32", "f64_plain", "f32_plain", "f32_split"])
@pytest.mark.parametrize("n", [8, 16, 24, 32, 48, 64, 96])
def test_solve_matches_oracle_fft_conv(prec, n):
    rho = inputs.make_density(n, 6, 300 + n, sigma=(0.03, 0.1), noise=1e-3)
    got, rho_used, _ = gpu_solve(rho, prec)
    ref = oracle.fft_conv(rho_used, 1.0 / n)
    l2, mx = _report(f"n={n} {prec}", got, ref)
    assert l2 <= TOL[prec]


# lengths with factors 3^2 and 5 (radix-5 and repeated radix-3 stages)
_SMOOTH_REF = {}


@pytest.mark.parametrize("prec", ["f64", "f32", "f64_plain", "f32_plain", "f32_split"])
@pytest.mark.parametrize("n", [40, 72, 80, 120, 144, 160, 200])
def test_five_smooth_sizes_match_oracle(prec, n):
    # radices 5, 3 x 3, 10, 15, 6, 20, 5 x 5
    rho = inputs.make_density(n, 8, 700 + n, sigma=(0.03, 0.1), noise=1e-3)
    got, rho_used, s = gpu_solve(rho, prec)
    assert s.info()["radices"][0] == 16
    key = (n, prec.startswith("f64"))
    if key not in _SMOOTH_REF:
        _SMOOTH_REF[key] = oracle.fft_conv(rho_used, 1.0 / n)
    l2, mx = _report(f"n={n} {prec}", got, _SMOOTH_REF[key])
    assert l2 <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [192, 216, 240, 288, 320, 360, 384, 400, 432, 480])
def test_five_smooth_large_sampled_direct_sum(prec, n):
    rho = inputs.make_density(n, 24, 800 + n, sigma=(0.01, 0.05), noise=1e-3)
    got, rho_used, s = gpu_solve(rho, prec)
    cells = _sample_cells(n, 16, n)
    ref = oracle.direct_sum_cells(rho_used, cells, 1.0 / n)
    g = got[cells[:, 0], cells[:, 1], cells[:, 2]]
    err = np.abs(g - ref).max() / np.abs(ref).max()
    print(f"n={n} {prec} radices {s.info()['radices']} variants {s.info()['variant']}: sampled rel max err {err:.3e}",
          flush=True)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f64_plain", "f32_plain"])
def test_blobs32_matches_direct_sum(prec):
    rho = inputs.workload_density("blobs32")
    got, rho_used, _ = gpu_solve(rho, prec)
    ref = oracle.direct_sum(rho_used, 1.0 / 32)
    l2, mx = _report(f"blobs32 {prec} vs direct sum", got, ref)
    assert l2 <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_nonunit_G_dx_self(prec):
    n = 24
    rho = inputs.make_density(n, 4, 77, sigma=(0.04, 0.1))
    dx, G, sc = 0.37, 6.674e-3, 2.3800774
    got, rho_used, _ = gpu_solve(rho, prec, dx=dx, G=G, self_coeff=sc)
    ref = oracle.fft_conv(rho_used, dx, G=G, self_coeff=sc)
    l2, _ = _report(f"n={n} {prec} G/dx/self", got, ref)
    assert l2 <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_impulse_response_on_gpu(prec):
    # a unit point mass gives phi[i] = G K(i - c): no oracle involved
    n = 32
    dx = 1.0 / n
    c = (5, 17, 30)
    rho = np.zeros((n, n, n))
    rho[c] = 1.0 / dx ** 3
    got, _, _ = gpu_solve(rho, prec)
    iz, iy, ix = np.indices((n, n, n))
    d = np.sqrt((iz - c[0]) ** 2 + (iy - c[1]) ** 2 + (ix - c[2]) ** 2)
    with np.errstate(divide="ignore"):
        k = np.where(d > 0, -1.0 / (dx * d), -2.38 / dx)
    l2, mx = _report(f"impulse {prec}", got, k)
    assert mx <= (1e-12 if prec == "f64" else 2e-6)


def test_linearity_and_determinism_on_gpu():
    n = 48
    r1 = inputs.make_density(n, 5, 1, sigma=(0.03, 0.08))
    r2 = np.random.default_rng(2).uniform(0, 1, (n, n, n))
    s = S.Solver(n, 1.0 / n, "f64")
    t1 = torch.from_numpy(r1).cuda()
    t2 = torch.from_numpy(r2).cuda()
    p1 = s(t1)
    p1b = s(t1)
    p2 = s(t2)
    pl = s((2.0 * t1 - 3.0 * t2).contiguous())
    torch.cuda.synchronize()
    assert torch.equal(p1, p1b)
    assert oracle.rel_l2(pl.cpu().numpy(), (2 * p1 - 3 * p2).cpu().numpy()) <= 1e-13
    # reciprocity <rho1, phi[rho2]> = <rho2, phi[rho1]>
    a = float((t1 * p2).sum())
    b = float((t2 * p1).sum())
    assert abs(a - b) <= 1e-12 * abs(a)


# ---------------------------------------------------------------------------
# Larger configurations: full oracle where it fits, sampled direct sums beyond
# ---------------------------------------------------------------------------

def _sample_cells(n, k, seed):
    rng = np.random.default_rng(seed)
    cells = rng.integers(0, n, (k, 3))
    corners = [[0, 0, 0], [n - 1, n - 1, n - 1], [0, n - 1, 0], [n - 1, 0, n - 1], [n // 2, n // 2, n // 2]]
    cells[:len(corners)] = corners
    return cells


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_n128_full_oracle(prec):
    n = 128
    rho = inputs.make_density(n, 32, 1128, sigma=(0.01, 0.05), noise=1e-3)
    got, rho_used, _ = gpu_solve(rho, prec)
    ref = oracle.fft_conv(rho_used, 1.0 / n)
    l2, mx = _report(f"n=128 {prec}", got, ref)
    assert l2 <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f64_plain", "f32_plain", "f32_split"])
def test_blobs256_sampled_direct_sum(prec):
    rho = inputs.workload_density("blobs256")
    got, rho_used, _ = gpu_solve(rho, prec)
    cells = _sample_cells(256, 96, 7)
    ref = oracle.direct_sum_cells(rho_used, cells, 1.0 / 256)
    g = got[cells[:, 0], cells[:, 1], cells[:, 2]]
    err = np.abs(g - ref).max() / np.abs(ref).max()
    print(f"blobs256 {prec}: sampled rel max err {err:.3e}", flush=True)
    assert err <= TOL[prec]


# ---------------------------------------------------------------------------
# Kernel variants: every variant of every pass gives the same solve
# ---------------------------------------------------------------------------

_BLOBS512 = {}


def _blobs512():
    if "rho" not in _BLOBS512:
        _BLOBS512["rho"] = inputs.workload_density("blobs512")
    return _BLOBS512["rho"]


@pytest.mark.parametrize("prec", ["f32", "f64", "f32_split"])
def test_blobs512_sampled_direct_sum(prec):
    # the benchmark's workload and launch configuration (library default variants)
    n = 512
    s = S.Solver(n, 1.0 / n, prec)
    rho = torch.from_numpy(_blobs512()).to("cuda", _dtype(prec))
    phi = s(rho)
    cells = _sample_cells(n, 24, 5)
    idx = torch.from_numpy(cells).to("cuda", torch.long)
    got = phi[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
    ref = oracle.direct_sum_cells(rho.double().cpu().numpy(), cells, 1.0 / n)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"blobs512 {prec} variants {s.info()['variant']}: sampled rel max err {err:.3e}", flush=True)
    assert err <= TOL[prec]
    del s, rho, phi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [256, 360, 400, 512])
def test_half_lds_y_exchange(prec, n):
    # the y passes exchanging through half the LDS in two rounds (both plan
    # families) against the one-round passes
    rho_np = inputs.make_density(n, 12, 7100 + n, sigma=(0.02, 0.06), noise=1e-3)
    s = S.Solver(n, 1.0 / n, prec)
    rho = torch.from_numpy(rho_np).to("cuda", _dtype(prec))
    S.ps_plan_set_variant(s.plan, 1, 0)
    S.ps_plan_set_variant(s.plan, 3, 0)
    base = s(rho)
    for yf, yi in ((6, 6), (7, 7), (6, 7), (7, 6)):
        S.ps_plan_set_variant(s.plan, 1, yf)
        S.ps_plan_set_variant(s.plan, 3, yi)
        got = s(rho)
        again = s(rho)
        l2 = float((got - base).norm() / base.norm())
        print(f"n={n} {prec} y variants {yf}/{yi}: relL2 vs one-round exchange {l2:.2e}", flush=True)
        assert torch.equal(got, again)
        assert l2 <= (1e-13 if prec == "f64" else 5e-7)
    del s, rho, base
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [256, 320, 400, 432, 480, 512])
def test_half_lds_z_exchange(prec, n):
    # the z pass exchanging through half the LDS in two rounds (both tile
    # widths) against the one-round wave-owned pass, and at n = 256 against
    # sampled direct sums
    rho_np = inputs.make_density(n, 12, 7000 + n, sigma=(0.02, 0.06), noise=1e-3)
    s = S.Solver(n, 1.0 / n, prec)
    rho = torch.from_numpy(rho_np).to("cuda", _dtype(prec))
    S.ps_plan_set_variant(s.plan, 2, 1)
    S.ps_plan_set_variant(s.plan, 6, 0)
    base = s(rho)
    ran = 0
    for zmode in (5,):
        S.ps_plan_set_variant(s.plan, 2, zmode)
        for zt in (0, 1):
            S.ps_plan_set_variant(s.plan, 6, zt)
            got = s(rho)
            again = s(rho)
            l2 = float((got - base).norm() / base.norm())
            print(f"n={n} {prec} zmode {zmode} ztile {zt}: relL2 vs one-round exchange {l2:.2e}", flush=True)
            assert torch.equal(got, again)
            assert l2 <= (1e-13 if prec == "f64" else 5e-7)
            ran += 1
    assert ran == 2
    if n == 256:
        S.ps_plan_set_variant(s.plan, 2, 5)
        S.ps_plan_set_variant(s.plan, 6, 0)
        got = s(rho).double().cpu().numpy()
        cells = _sample_cells(n, 24, 11)
        ref = oracle.direct_sum_cells(rho.double().cpu().numpy(), cells, 1.0 / n)
        err = np.abs(got[cells[:, 0], cells[:, 1], cells[:, 2]] - ref).max() / np.abs(ref).max()
        assert err <= TOL[prec]
    del s, rho, base
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_persistent_z_pass_n512(prec):
    # the persistent prefetching z pass against the one-tile-per-workgroup one
    n = 512
    s = S.Solver(n, 1.0 / n, prec)
    rho = torch.from_numpy(_blobs512()).to("cuda", _dtype(prec))
    S.ps_plan_set_variant(s.plan, 2, 2)
    base = s(rho).double()
    S.ps_plan_set_variant(s.plan, 2, 3)
    got = s(rho).double()
    again = s(rho).double()
    l2 = float((got - base).norm() / base.norm())
    print(f"n=512 {prec}: persistent z pass vs zmode 2 relL2 {l2:.2e}, bitwise {bool(torch.equal(got, base))}",
          flush=True)
    assert torch.equal(got, again)
    assert l2 <= (1e-13 if prec == "f64" else 5e-7)
    del s, rho, base, got, again
    torch.cuda.empty_cache()


def test_split_persistent_passes_n512():
    # the split form's persistent z and y passes against its one-tile-per-workgroup ones
    n = 512
    s = S.Solver(n, 1.0 / n, "f32_split")
    rho = torch.from_numpy(_blobs512()).to("cuda", torch.float32)
    for k in range(5):
        S.ps_plan_set_variant(s.plan, k, 0)
    base = s(rho).double()
    for k, v in ((2, 1), (2, 3), (2, 4), (1, 2), (3, 2)):
        S.ps_plan_set_variant(s.plan, k, v)
        got = s(rho).double()
        l2 = float((got - base).norm() / base.norm())
        print(f"n=512 f32_split pass {k} variant {v}: relL2 vs variant 0 {l2:.2e}", flush=True)
        assert l2 <= 5e-7
    del s, rho, base, got
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_variants_agree_n256(prec):
    n = 256
    rho_np = inputs.make_density(n, 16, 99, sigma=(0.02, 0.06), noise=1e-3)
    s = S.Solver(n, 1.0 / n, prec)
    rho = torch.from_numpy(rho_np).to("cuda", _dtype(prec))
    for k in range(5):
        S.ps_plan_set_variant(s.plan, k, 0)
    base = s(rho).double().cpu().numpy()
    tol = 1e-13 if prec == "f64" else 5e-7
    for k, nv in zip(range(5), (6, 8, 6, 8, 6)):
        for v in range(1, nv):
            try:
                S.ps_plan_set_variant(s.plan, k, v)
            except S.PSError:
                # half-LDS z and y exchanges: not split
                assert ((k == 2 and v == 5) or (k in (1, 3) and v >= 6)) and prec == "f32_split"
                continue
            got = s(rho).double().cpu().numpy()
            l2 = oracle.rel_l2(got, base)
            print(f"n=256 {prec} pass {k} variant {v}: relL2 vs variant 0 = {l2:.2e}", flush=True)
            assert l2 <= tol
        S.ps_plan_set_variant(s.plan, k, 0)
    # all-defaults result against sampled direct sums
    for k, v in zip(range(5), (1, 1, 2, 1, 1)):
        S.ps_plan_set_variant(s.plan, k, v)
    got = s(rho).double().cpu().numpy()
    rho64 = rho.double().cpu().numpy()
    cells = _sample_cells(n, 48, 3)
    ref = oracle.direct_sum_cells(rho64, cells, 1.0 / n)
    err = np.abs(got[cells[:, 0], cells[:, 1], cells[:, 2]] - ref).max() / np.abs(ref).max()
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
@pytest.mark.parametrize("n", [16, 48, 96, 120])
@pytest.mark.parametrize("zmode", [0, 1, 3, 4])
@pytest.mark.parametrize("ztile", [0, 1])
def test_zmodes_match_oracle(prec, n, zmode, ztile):
    rho = inputs.make_density(n, 5, 500 + n, sigma=(0.03, 0.1), noise=1e-3)
    s = S.Solver(n, 1.0 / n, prec)
    S.ps_plan_set_variant(s.plan, 2, zmode)
    S.ps_plan_set_variant(s.plan, 6, ztile)
    r = torch.from_numpy(rho).to("cuda", _dtype(prec))
    got = s(r).double().cpu().numpy()
    ref = oracle.fft_conv(r.double().cpu().numpy(), 1.0 / n)
    l2, _ = _report(f"zmode {zmode} ztile {ztile} n={n} {prec}", got, ref)
    assert l2 <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [72, 144, 160, 192, 200, 216, 240, 288, 320, 360, 384, 400, 432, 480])
def test_two_stage_radix32_family(prec, n):
    # the two-stage plans (P = 288: 24 x 12, 320: 32 x 10, 384: 32 x 12,
    # 480: 32 x 15, 576: 24 x 24, 640: 32 x 20, 720: 24 x 30, 768: 32 x 24,
    # 800: 32 x 25, 864: 32 x 27, 960: 32 x 30; 144: 16 x 9, 400: 16 x 25,
    # 432: 16 x 27): every variant on that family agrees with the
    # radix-16-based plan to rounding, and the solve matches direct sums at
    # sampled cells
    rho_np = inputs.make_density(n, 12, 800 + n, sigma=(0.02, 0.06), noise=1e-3)
    s = S.Solver(n, 1.0 / n, prec)
    rho = torch.from_numpy(rho_np).to("cuda", _dtype(prec))
    for k in range(5):
        S.ps_plan_set_variant(s.plan, k, 0)
    base = s(rho).double()
    tol = 1e-13 if prec == "f64" else 5e-7
    for k, vs in ((0, (1, 3)), (1, (1, 3, 5)), (2, (2, 3)), (3, (1, 3, 5)), (4, (1, 3))):
        for v in vs:
            try:
                S.ps_plan_set_variant(s.plan, k, v)
            except S.PSError:
                continue  # a tile the LDS cannot hold
            err = float((s(rho).double() - base).norm() / base.norm())
            print(f"n={n} {prec} pass {k} variant {v}: relL2 vs radix-16 plan = {err:.2e}", flush=True)
            assert err <= tol, (k, v, err)
        S.ps_plan_set_variant(s.plan, k, 0)
    for k, v in ((0, 1), (1, 1), (2, 2), (3, 1), (4, 1)):
        S.ps_plan_set_variant(s.plan, k, v)
    got = s(rho).double().cpu().numpy()
    rho64 = rho.double().cpu().numpy()
    cells = _sample_cells(n, 6, 5)
    ref = oracle.direct_sum_cells(rho64, cells, 1.0 / n)
    err = np.abs(got[cells[:, 0], cells[:, 1], cells[:, 2]] - ref).max() / np.abs(ref).max()
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
@pytest.mark.parametrize("n", [24, 40, 120, 200])
def test_x_rows_match_oracle(prec, n):
    # 8, 16 and 32 rows per x-pass workgroup (ragged last y tiles at these n)
    rho = inputs.make_density(n, 5, 700 + n, sigma=(0.03, 0.1), noise=1e-3)
    s = S.Solver(n, 1.0 / n, prec)
    r = torch.from_numpy(rho).to("cuda", _dtype(prec))
    ref = oracle.fft_conv(r.double().cpu().numpy(), 1.0 / n)
    for v in (0, 2, 4):
        S.ps_plan_set_variant(s.plan, 0, v)
        S.ps_plan_set_variant(s.plan, 4, v)
        got = s(r).double().cpu().numpy()
        l2, _ = _report(f"x rows variant {v} n={n} {prec}", got, ref)
        assert l2 <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
@pytest.mark.parametrize("n", [40, 128, 192, 384])
def test_z_tile_widths_agree(prec, n):
    # a pencil's arithmetic does not depend on how many pencils share a
    # workgroup: both tile widths agree to rounding in every z form (not
    # always bitwise: the compiler may contract products into FMAs
    # differently in the two kernels)
    rho = inputs.make_density(n, 6, 900 + n, sigma=(0.03, 0.08), noise=1e-3)
    s = S.Solver(n, 1.0 / n, prec)
    r = torch.from_numpy(rho).to("cuda", _dtype(prec))
    for zmode in range(6):
        try:
            S.ps_plan_set_variant(s.plan, 2, zmode)
        except S.PSError:
            continue
        S.ps_plan_set_variant(s.plan, 6, 0)
        a = s(r).double()
        S.ps_plan_set_variant(s.plan, 6, 1)
        b = s(r).double()
        err = float((a - b).norm() / a.norm())
        assert err <= (1e-14 if prec == "f64" else 2e-7), (zmode, n, prec, err)


def test_persistent_z_fallback_where_lds_is_short():
    # FP64 at P = 960: the persistent z pass on the radix-16-based plan does
    # not fit in LDS, so variant 4 runs the wave-owned pass (the same kernel
    # as variant 1); variant 3 runs the radix-32-based plan's persistent form,
    # which fits, and agrees to rounding
    n = 480
    rho = inputs.make_density(n, 6, 4800, sigma=(0.02, 0.06), noise=1e-3)
    s = S.Solver(n, 1.0 / n, "f64")
    r = torch.from_numpy(rho).to("cuda", torch.float64)
    S.ps_plan_set_variant(s.plan, 2, 1)
    S.ps_plan_set_variant(s.plan, 6, 0)
    ref = s(r)
    S.ps_plan_set_variant(s.plan, 2, 4)
    assert torch.equal(s(r), ref)
    S.ps_plan_set_variant(s.plan, 2, 3)
    err = float((s(r) - ref).norm() / ref.norm())
    assert err <= 1e-13, err


def test_autotune_writes_cache(tmp_path):
    n = 64
    s = S.Solver(n, 1.0 / n, "f32")
    path = str(tmp_path / "tune.txt")
    S.ps_autotune(s.plan, torch.cuda.current_stream().cuda_stream, path)
    lines = open(path).read().split()
    assert lines[:2] == ["128", "f32"]
    chosen = s.info()["variant"], s.info()["z_tile"]
    s2 = S.Solver(n, 1.0 / n, "f32", tune_cache=path)
    assert (s2.info()["variant"], s2.info()["z_tile"]) == chosen
    assert len(open(path).read().split()) == 8  # P, precision, five variants, the z tile
    rho = inputs.make_density(n, 5, 7, sigma=(0.03, 0.1))
    r = torch.from_numpy(rho).to("cuda", torch.float32)
    got = s2(r).double().cpu().numpy()
    ref = oracle.fft_conv(r.double().cpu().numpy(), 1.0 / n)
    assert oracle.rel_l2(got, ref) <= 1e-6


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_autotune_n256_includes_half_lds_forms(prec, tmp_path):
    # at P = 512 the autotuner also times the half-LDS y and z forms; its
    # choice, read back from the cache, solves to rounding of the defaults
    n = 256
    s = S.Solver(n, 1.0 / n, prec)
    rho = torch.from_numpy(inputs.make_density(n, 8, 4242, sigma=(0.02, 0.06), noise=1e-3)).to("cuda", _dtype(prec))
    base = s(rho)
    path = str(tmp_path / "tune.txt")
    S.ps_autotune(s.plan, torch.cuda.current_stream().cuda_stream, path)
    fields = open(path).read().split()
    assert fields[:2] == ["512", prec] and len(fields) == 8
    s2 = S.Solver(n, 1.0 / n, prec, tune_cache=path)
    assert (s2.info()["variant"], s2.info()["z_tile"]) == (s.info()["variant"], s.info()["z_tile"])
    got = s2(rho)
    l2 = float((got - base).norm() / base.norm())
    print(f"n=256 {prec} autotuned {s2.info()['variant']} z tile {s2.info()['z_tile']}: relL2 vs defaults {l2:.2e}",
          flush=True)
    assert l2 <= (1e-13 if prec == "f64" else 5e-7)
    del s, s2, rho, base, got
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# Split-bf16 matrix-core DFT-16: the six-term form meets the single-precision
# bound; the three-term form is reported (it is the labelled, less accurate
# reading of "3-term split-BF16")
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [32, 64, 128])
def test_split_terms_error(n):
    rho = inputs.make_density(n, 24, 700 + n, sigma=(0.01, 0.05), noise=1e-3)
    r = torch.from_numpy(rho).to("cuda", torch.float32)
    ref = oracle.fft_conv(r.double().cpu().numpy(), 1.0 / n)
    s = S.Solver(n, 1.0 / n, "f32_split")
    errs = {}
    for terms in (6, 3):
        S.ps_plan_set_variant(s.plan, 5, terms)
        got = s(r).double().cpu().numpy()
        errs[terms] = _report(f"split {terms} terms n={n}", got, ref)
    assert errs[6][0] <= 1e-6
    assert errs[3][0] <= 5e-5
    # the six-term products carry more of the operands than the three-term ones
    assert errs[6][0] < errs[3][0]


@pytest.mark.parametrize("prec", ["f32", "f32_split"])
def test_blobs512_full_field_vs_f64_path(prec):
    # the whole 512^3 field of the single-precision paths against the FP64
    # path (itself within 1e-12 of the oracle at every size tested), in the
    # launch configuration the benchmark times
    n = 512
    rho64 = _blobs512()
    s64 = S.Solver(n, 1.0 / n, "f64")
    s = S.Solver(n, 1.0 / n, prec)
    r32 = torch.from_numpy(rho64).to("cuda", torch.float32)
    ref = s64(r32.double())
    got = s(r32).double()
    l2 = float((got - ref).norm() / ref.norm())
    mx = float((got - ref).abs().max() / ref.abs().max())
    print(f"512^3 full field {prec} vs f64 path: relL2={l2:.3e} relMax={mx:.3e}", flush=True)
    assert l2 <= 1e-6
    del s64, s, r32, ref, got
    torch.cuda.empty_cache()
