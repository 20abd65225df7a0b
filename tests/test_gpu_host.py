"""GPU tests of host-resident solves (ps_solve_host): the staged, overlapped
upload / solve / download sequence must give every solve exactly what
ps_solve gives on the same density already in device memory, with pinned and
with pageable host arrays, for sequences shorter and longer than the two
staging slots.
"""
import numpy as np
import pytest

from conftest import gpu_available
from paper_2409_02294_amd import inputs

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_2409_02294_amd import solver as S


def _densities(n, count, seed, dtype):
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        blobs = inputs.draw_blobs(rng, int(rng.integers(4, 17)), centre=(0.1, 0.9), sigma=(0.03, 0.08))
        out.append(torch.from_numpy(inputs.blob_density(n, blobs)).to(dtype))
    return out


@pytest.mark.parametrize("prec", ["f32", "f64", "f32_split", "f64_plain"])
@pytest.mark.parametrize("pinned", [True, False])
@pytest.mark.parametrize("count", [1, 2, 5])
def test_host_solves_match_device_solves(prec, pinned, count):
    n = 48
    s = S.Solver(n, 1.0 / n, prec)
    rhos = _densities(n, count, 6000 + count, s.dtype)
    if pinned:
        rhos = [r.pin_memory() for r in rhos]
    outs = [torch.empty_like(r).pin_memory() if pinned else torch.empty_like(r) for r in rhos]
    s.solve_host(rhos, outs)
    for r, o in zip(rhos, outs):
        ref = s(r.to("cuda")).cpu()
        assert torch.equal(o, ref)


def test_host_solves_repeat_with_other_arrays():
    # the plan's copy streams and events are reused across calls
    n = 64
    s = S.Solver(n, 1.0 / n, "f32")
    stage = torch.empty(S.ps_host_stage_bytes(s.plan), dtype=torch.uint8, device="cuda")
    a = [r.pin_memory() for r in _densities(n, 3, 6100, torch.float32)]
    b = [r.pin_memory() for r in _densities(n, 4, 6200, torch.float32)]
    oa = s.solve_host(a, stage=stage)
    ob = s.solve_host(b, stage=stage)
    for r, o in zip(a + b, oa + ob):
        assert torch.equal(o, s(r.to("cuda")).cpu())


def test_plan_lifecycle_with_streams():
    # plans that own batch and copy streams are created and destroyed repeatedly
    for it in range(6):
        sizes = [32, 48, 64]
        solvers = [S.Solver(n, 1.0 / n, "f32") for n in sizes]
        rhos = [d.to("cuda") for d in (_densities(n, 1, 6300 + it * 10 + n, torch.float32)[0] for n in sizes)]
        outs = S.solve_batched(solvers, rhos)
        host = [r.cpu().pin_memory() for r in rhos]
        back = [solvers[k].solve_host([host[k]])[0] for k in range(len(sizes))]
        for s, r, o, b in zip(solvers, rhos, outs, back):
            ref = s(r)
            assert torch.equal(o, ref) and torch.equal(b, ref.cpu())
        for s in solvers:
            s.close()
    torch.cuda.synchronize()


def test_two_plans_on_two_streams():
    # plans own their workspaces: solves of two plans may run concurrently
    n = 64
    a, b = S.Solver(n, 1.0 / n, "f32"), S.Solver(n, 1.0 / n, "f64")
    ra = _densities(n, 1, 6400, torch.float32)[0].to("cuda")
    rb = _densities(n, 1, 6401, torch.float64)[0].to("cuda")
    ref_a, ref_b = a(ra), b(rb)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs_a, outs_b = [], []
    for _ in range(4):
        with torch.cuda.stream(s1):
            outs_a.append(a(ra))
        with torch.cuda.stream(s2):
            outs_b.append(b(rb))
    torch.cuda.synchronize()
    for oa, ob in zip(outs_a, outs_b):
        assert torch.equal(oa, ref_a) and torch.equal(ob, ref_b)


@pytest.mark.parametrize("prec", ["f64", "f32", "f32_split", "f64_plain", "f32_plain"])
def test_host_solves_match_oracle(prec):
    # every solve of a host-resident sequence against the FP64 oracle's FFT
    # convolution of the same (precision-rounded) density
    import oracle
    n = 40
    tol = 1e-12 if prec.startswith("f64") else 1e-6
    s = S.Solver(n, 1.0 / n, prec)
    rhos = [r.pin_memory() for r in _densities(n, 3, 6500, s.dtype)]
    outs = s.solve_host(rhos)
    torch.cuda.synchronize()
    for r, o in zip(rhos, outs):
        ref = oracle.fft_conv(r.double().numpy(), 1.0 / n)
        got = o.double().numpy()
        l2, mx = oracle.rel_l2(got, ref), oracle.rel_max(got, ref)
        print(f"host {prec}: relL2={l2:.3e} relMax={mx:.3e}", flush=True)
        assert l2 <= tol
