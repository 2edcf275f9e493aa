"""tg_nsdf_query_noalloc (images in the library's static device array) against tg_nsdf_query
(images in the handle's buffer), through the C ABI.

Both run the same kernels on the same inputs, so the bar is bit-for-bit equality of the network
outputs and input gradients.  Two calls in a row go through the static array, the second with
fewer objects and fewer points than the first (what the first left behind must not leak into
it); a handle with more objects than the array holds is rejected before anything is launched.
"""
import numpy as np
import pytest

from paper_2606_22332_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def grouped_points(counts, seed):
    rng = np.random.default_rng(seed)
    offs = np.zeros(len(counts) + 1, np.int64)
    offs[1:] = np.cumsum(counts)
    x = rng.uniform(-1.0, 1.0, (int(offs[-1]), 3)).astype(np.float32)
    return offs, x


def test_noalloc_query_equals_query_on_two_calls(torch_cuda):
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    grids = synth.make_scene("c2", num_envs=4, num_steps=2).grids          # 8 objects
    cases = [(grids, [700, 0, 1201, 64, 333, 1, 900, 517], 21),            # ragged, one empty object
             (grids[:3], [129, 40, 250], 22)]                               # fewer objects, fewer points
    results = []
    handles = []
    for gs, counts, seed in cases:
        ns = B.Nsdf(gs)
        handles.append(ns)
        P = torch.from_numpy(synth.nsdf_init(len(gs), seed)).cuda()
        offs, x = grouped_points(counts, seed)
        xd = torch.from_numpy(x).cuda()
        out = torch.full((x.shape[0],), float("nan"), device="cuda")
        g = torch.full((x.shape[0], 3), float("nan"), device="cuda")
        print(f"noalloc call: {len(gs)} objects, {x.shape[0]} points", flush=True)
        ns.query(P, offs, xd, noalloc=True, out=out, grad_out=g)
        results.append((ns, P, offs, xd, out, g))
    torch.cuda.synchronize()
    for ns, P, offs, xd, out, g in results:        # the handle-buffer path on the same inputs
        ref_out, ref_g = ns.query(P, offs, xd)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all() and torch.isfinite(g).all()
        assert torch.equal(out, ref_out)
        assert torch.equal(g, ref_g)
    for ns in handles:
        ns.close()


def test_noalloc_query_rejects_more_objects_than_the_array_holds(torch_cuda):
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    n = 4
    vals = np.zeros((n, n, n), np.float32)
    g = synth.Grid(n, np.zeros(3, np.float32), np.float32(0.01), vals, "custom", {})
    ns = B.Nsdf([g] * 65)
    P = torch.zeros((65, 15681), device="cuda")
    offs = np.zeros(66, np.int64)
    offs[1:] = np.arange(1, 66)
    xd = torch.zeros((65, 3), device="cuda")
    out = torch.full((65,), float("nan"), device="cuda")
    with pytest.raises(B.TgError, match="exceed the static scratch"):
        ns.query(P, offs, xd, grad=False, noalloc=True, out=out)
    torch.cuda.synchronize()
    assert torch.isnan(out).all()                  # nothing was launched
    ns.close()
