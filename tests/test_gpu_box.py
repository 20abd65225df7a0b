"""GPU parity of solves on boxes of nx x ny x nz cells (ps_plan_create_box)
against the FP64 oracle's box routines: whole solves against its FFT
convolution at several shapes and spacings in every pruned precision, every
pass against numpy on a box, sampled direct sums on large boxes, equal
lengths against the cubic plan, batches mixing boxes and cubes, and
host-resident box solves.  Arrays are [z][y][x].
"""
import numpy as np
import pytest

import oracle
from conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_2409_02294_amd import solver as S

TOL = {"f64": 1e-12, "f32": 1e-6, "f32_split": 1e-6}


def _dtype(prec):
    return torch.float64 if prec.startswith("f64") else torch.float32


def _box_density(shape, seed, blobs=4):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny, (np.arange(nx) + 0.5) / nx,
                          indexing="ij")
    rho = np.zeros(shape)
    for _ in range(blobs):
        c = rng.uniform(0.2, 0.8, 3)
        s = rng.uniform(0.05, 0.12)
        rho += rng.uniform(0.5, 2.0) * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * s * s))
    return rho + 1e-3 * rng.uniform(0, 1, shape)


def _solve(rho_np, prec, dx, dy, dz, G=1.0):
    nz, ny, nx = rho_np.shape
    s = S.Solver((nx, ny, nz), dx, prec, G=G, spacing=(dy, dz))
    rho = torch.from_numpy(np.ascontiguousarray(rho_np)).to("cuda", _dtype(prec))
    phi = s(rho)
    torch.cuda.synchronize()
    return phi.double().cpu().numpy(), rho.double().cpu().numpy(), s


SHAPES = [((32, 48, 16), (1 / 32, 1 / 32, 1 / 32)), ((40, 24, 64), (0.025, 0.03, 0.02)),
          ((16, 8, 96), (1 / 16, 1 / 16, 1 / 96)), ((96, 72, 40), (0.01, 0.012, 0.02)),
          ((8, 128, 24), (0.1, 0.008, 0.05)), ((120, 16, 48), (1 / 120, 1 / 120, 1 / 120))]


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
@pytest.mark.parametrize("dims,sp", SHAPES)
def test_box_solve_matches_oracle(prec, dims, sp):
    nx, ny, nz = dims
    rho = _box_density((nz, ny, nx), nx + 3 * ny + 7 * nz)
    got, used, s = _solve(rho, prec, *sp, G=0.8)
    info = s.info()
    assert (info["nx"], info["ny"], info["nz"]) == dims
    ref = oracle.fft_conv_box(used, *sp, G=0.8)
    l2, mx = oracle.rel_l2(got, ref), oracle.rel_max(got, ref)
    print(f"box {dims} {prec}: relL2={l2:.3e} relMax={mx:.3e}", flush=True)
    assert l2 <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dims", [(40, 24, 16), (32, 64, 48)])
def test_box_passes_match_numpy(prec, dims):
    # every pass on a box against numpy, in the layouts between the passes
    nx, ny, nz = dims
    px, py, pz = 2 * nx, 2 * ny, 2 * nz
    hx = nx + 1
    hpx = (hx + 15) // 16 * 16
    rng = np.random.default_rng(sum(dims))
    dt = _dtype(prec)
    cdt = torch.complex128 if dt == torch.float64 else torch.complex64
    tol = 1e-13 if prec == "f64" else 2e-6
    s = S.Solver(dims, 1.0 / nx, prec)
    st = torch.cuda.current_stream().cuda_stream

    def run(pass_id, x_np, out_shape, out_complex):
        x = torch.from_numpy(x_np).to("cuda")
        x = x.to(cdt if np.iscomplexobj(x_np) else dt).contiguous()
        out = torch.empty(out_shape, dtype=cdt if out_complex else dt, device="cuda")
        S.ps_debug_pass(s.plan, pass_id, x.data_ptr(), out.data_ptr(), st)
        torch.cuda.synchronize()
        return x.cpu().numpy().astype(np.complex128 if np.iscomplexobj(x_np) else np.float64), out.cpu().numpy()

    def check(tag, got, ref):
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"box pass {tag} {dims} {prec}: rel max err {err:.2e}", flush=True)
        assert err <= tol

    rho = rng.uniform(-1, 1, (nz, ny, nx))
    rin, t1 = run(0, rho, (hx, nz, ny), True)
    check("x_r2c", t1, np.transpose(np.fft.rfft(rin, n=px, axis=2), (2, 0, 1)))
    a = rng.standard_normal((hx, nz, ny)) + 1j * rng.standard_normal((hx, nz, ny))
    ain, t2 = run(1, a, (hx, py, nz), True)
    check("y_fwd", t2, np.transpose(np.fft.fft(ain, n=py, axis=2), (0, 2, 1)))
    b = rng.standard_normal((hx, py, nz)) + 1j * rng.standard_normal((hx, py, nz))
    bin_, t3 = run(2, b, (hx, nz, py), True)
    g = oracle.fft3_box(oracle.kernel_pad_box(nx, ny, nz, 1.0 / nx, 1.0 / nx, 1.0 / nx)).real  # [kz][ky][kx]
    g = np.transpose(g, (2, 1, 0))[:hx] * ((1.0 / nx) ** 3 / (px * py * pz))                    # [kx][ky][kz]
    ref = np.fft.ifft(np.fft.fft(bin_, n=pz, axis=2) * g, axis=2)[:, :, :nz] * pz
    check("z_conv", t3, np.transpose(ref, (0, 2, 1)))
    c = rng.standard_normal((hx, nz, py)) + 1j * rng.standard_normal((hx, nz, py))
    cin, t4 = run(3, c, (nz, ny, hpx), True)
    check("y_inv", t4[:, :, :hx], np.transpose(np.fft.ifft(cin, axis=2)[:, :, :ny] * py, (1, 2, 0)))
    d = rng.standard_normal((nz, ny, hpx)) + 1j * rng.standard_normal((nz, ny, hpx))
    d[:, :, hx:] = 1e30
    din, out = run(4, d, (nz, ny, nx), False)
    check("x_c2r", out, np.fft.irfft(din[:, :, :hx], n=px, axis=2)[:, :, :nx] * px)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dims", [(512, 256, 128), (128, 512, 256), (256, 128, 512)])
def test_large_box_sampled_direct_sum(prec, dims):
    nx, ny, nz = dims
    dx = 1.0 / 512
    rho = _box_density((nz, ny, nx), 17 + nx // 128, blobs=12)
    got, used, _ = _solve(rho, prec, dx, dx, dx)
    rng = np.random.default_rng(3)
    cells = np.stack([rng.integers(0, nz, 12), rng.integers(0, ny, 12), rng.integers(0, nx, 12)], axis=1)
    cells[:2] = [[0, 0, 0], [nz - 1, ny - 1, nx - 1]]
    ref = oracle.direct_sum_cells_box(used, cells, dx, dx, dx)
    g = got[cells[:, 0], cells[:, 1], cells[:, 2]]
    err = np.abs(g - ref).max() / np.abs(ref).max()
    print(f"box {dims} {prec}: sampled rel max err {err:.3e}", flush=True)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split"])
def test_box_entry_with_equal_lengths_is_the_cubic_plan(prec):
    n = 48
    rho = torch.from_numpy(_box_density((n, n, n), 5)).to("cuda", _dtype(prec))
    a = S.Solver(n, 1.0 / n, prec, spacing=(1.5 / n, 0.5 / n))
    h = S.ps_plan_create_box(n, n, n, 1.0 / n, 1.5 / n, 0.5 / n, S.PRECISIONS[prec])
    try:
        assert S.ps_plan_query(h)["variant"] == a.info()["variant"]
        assert S.ps_plan_workspace_bytes(h) == S.ps_plan_workspace_bytes(a.plan)
    finally:
        S.ps_plan_destroy(h)
    b = S.Solver((n, n, n), 1.0 / n, prec, spacing=(1.5 / n, 0.5 / n))
    assert torch.equal(a(rho), b(rho))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_box_variants_agree(prec):
    # every variant a box plan may run gives the same result to rounding
    dims = (256, 256, 32)  # x and y lengths with the radix-32-based family, z without
    rho = torch.from_numpy(_box_density((32, 256, 256), 9)).to("cuda", _dtype(prec))
    s = S.Solver(dims, 1.0 / 256, prec)
    ref = s(rho).double()
    tol = 1e-13 if prec == "f64" else 1e-6
    for pass_id, variants in ((0, (0, 1)), (1, (0, 1)), (2, (0, 1)), (3, (0, 1)), (4, (0, 1)), (6, (0, 1))):
        for v in variants:
            t = S.Solver(dims, 1.0 / 256, prec)
            S.ps_plan_set_variant(t.plan, pass_id, v)
            err = float((t(rho).double() - ref).norm() / ref.norm())
            assert err <= tol, (pass_id, v, err)
            t.close()
    for pass_id, v in ((1, 2), (3, 3), (2, 3), (2, 4), (2, 2)):
        with pytest.raises(S.PSError):
            S.ps_plan_set_variant(s.plan, pass_id, v)


def test_batch_of_boxes_and_cubes_equals_single_solves():
    dims = [(32, 48, 16), (48, 48, 48), (32, 48, 16), (16, 16, 40), (64, 32, 32)]
    solvers = [S.Solver(d, 1.0 / d[0], "f32") for d in dims]
    rhos = [torch.from_numpy(_box_density((d[2], d[1], d[0]), 50 + k)).to("cuda", torch.float32)
            for k, d in enumerate(dims)]
    outs = S.solve_batched(solvers, rhos)
    for s, r, o in zip(solvers, rhos, outs):
        assert torch.equal(o, s(r))


def test_host_resident_box_solves():
    dims = (40, 24, 64)
    s = S.Solver(dims, 1.0 / 40, "f32")
    rhos = [torch.from_numpy(_box_density((64, 24, 40), 70 + k)).to(torch.float32).pin_memory() for k in range(3)]
    outs = s.solve_host(rhos)
    for r, o in zip(rhos, outs):
        ref = oracle.fft_conv_box(r.double().numpy(), 1 / 40, 1 / 40, 1 / 40)
        assert oracle.rel_l2(o.double().numpy(), ref) <= 1e-6
        assert torch.equal(o, s(r.to("cuda")).cpu())
