"""The readout's C ABI under the ways a caller drives it (include/tg_readout.h, conventions):
a step captured into the caller's own HIP graph, two handles on two streams at once, misaligned
buffers rejected before anything is launched, and handles created and destroyed in a loop
without leaking device memory.  Results are compared with plain eager calls of the same library,
bit for bit (the same kernels on the same inputs)."""
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


def snapshot(out):
    return {k: v.clone() for k, v in out.items()}


def assert_same(a, b):
    import torch
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_step_captured_in_a_caller_graph(torch_cuda):
    """tg_readout_step recorded into a torch CUDA graph: every replay equals an eager step from
    the same noise state (replays 1 and 2 continue the state like two eager steps; a reset between
    replays starts it over), with eager work and synchronisations between the replays."""
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    sc = synth.make_scene("c2", num_envs=40, num_steps=2)
    inp = synth.make_inputs(sc)
    d = B.to_device(inp)
    ro = B.Readout(sc)
    ro.alloc_outputs(1)
    ro.reset(None, 0)
    ro.step(d, 0, s_out=0)
    torch.cuda.synchronize()
    e0 = snapshot(ro.out)
    ro.step(d, 0, s_out=0)            # same step index again: the noise state has moved on
    torch.cuda.synchronize()
    e1 = snapshot(ro.out)
    assert not torch.equal(e0["ft_noisy"], e1["ft_noisy"])
    ro.reset(None, 0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ro.step(d, 0, s_out=0)
    for k in ro.out:
        ro.out[k].fill_(7)
    torch.cuda.synchronize()
    expected = [e0, e1, e0]
    for i, exp in enumerate(expected):
        if i == 2:
            ro.reset(None, 0)
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(4096, device="cuda").sum().item()   # eager work between replays
        assert np.isfinite(junk)
        assert_same(exp, ro.out)
    del g
    ro.close()


def test_two_handles_on_two_streams(torch_cuda):
    """Two handles (different scenes and noise seeds) rolled out at the same time on two streams
    give what each gives alone on the default stream."""
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    scenes = [synth.make_scene("c2", num_envs=64, num_steps=5), synth.make_scene("c3", num_envs=24, num_steps=5)]
    inps = [synth.make_inputs(sc) for sc in scenes]
    alone = []
    for sc, inp in zip(scenes, inps):
        ro = B.Readout(sc)
        ro.alloc_outputs(5)
        ro.rollout(B.to_device(inp), 5)
        torch.cuda.synchronize()
        alone.append(snapshot(ro.out))
        ro.close()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ros, ds = [], []
    for sc, inp in zip(scenes, inps):
        ro = B.Readout(sc)
        ro.alloc_outputs(5)
        ros.append(ro)
        ds.append(B.to_device(inp))
    torch.cuda.synchronize()
    for _ in range(2):                 # the second round replays the handles' cached graphs
        for ro, d, st in zip(ros, ds, streams):
            ro.reset(None, 0, stream=st)
            ro.rollout(d, 5, stream=st)
        torch.cuda.synchronize()
        for ro, ref in zip(ros, alone):
            assert_same(ref, ro.out)
    for ro in ros:
        ro.close()


def test_misaligned_buffers_are_rejected(torch_cuda):
    """Inputs and outputs off their 16-byte alignment: TG_ERR_INVALID_ARGUMENT with a message, and
    nothing launched (the outputs keep their fill)."""
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    sc = synth.make_scene("c2", num_envs=8, num_steps=1)
    inp = synth.make_inputs(sc)
    d = B.to_device(inp)
    ro = B.Readout(sc)
    ro.alloc_outputs(1)
    for k in ro.out:
        ro.out[k].fill_(3)
    torch.cuda.synchronize()
    # a link-state buffer that starts one float late
    ls = torch.zeros(d.link_state.numel() + 4, dtype=torch.float32, device="cuda")
    bad = B.to_device(inp)
    bad.link_state = ls[1:1 + d.link_state.numel()].view_as(d.link_state)
    with pytest.raises(B.TgError, match="misaligned|aligned"):
        ro.step(bad, 0)
    # a depth output that starts one float late
    good_depth = ro.out["depth"]
    buf = torch.full((good_depth.numel() + 4,), 3.0, dtype=torch.float32, device="cuda")
    ro.out["depth"] = buf[1:1 + good_depth.numel()].view_as(good_depth)
    with pytest.raises(B.TgError, match="misaligned|aligned"):
        ro.step(d, 0)
    torch.cuda.synchronize()
    assert torch.all(buf == 3.0)
    ro.out["depth"] = good_depth
    for k, v in ro.out.items():
        assert torch.all(v == 3), k    # nothing was launched: the fill is untouched
    ro.step(d, 0)                      # the aligned call still works
    torch.cuda.synchronize()
    ro.close()


def test_create_destroy_loop_does_not_leak(torch_cuda):
    """Handles created, used once and destroyed in a loop (noisy grid and thermal configurations):
    after a warm-up (the runtime loads code objects and sets up its pools on first use), forty more
    create / rollout / destroy cycles leave the device's free memory where it was."""
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    scenes = [synth.make_scene("c2", num_envs=32, num_steps=2), synth.make_scene("c5", num_envs=4, num_steps=2)]
    inps = [synth.make_inputs(sc) for sc in scenes]
    ds = [B.to_device(inp) for inp in inps]
    outs = []
    for sc in scenes:                  # caller-owned outputs, allocated once outside the loop
        ro = B.Readout(sc)
        outs.append(ro.alloc_outputs(2))
        ro.out = {}
        ro.close()

    def cycle(i):
        ro = B.Readout(scenes[i % 2])
        ro.out = outs[i % 2]
        ro.rollout(ds[i % 2], 2)
        torch.cuda.synchronize()
        ro.out = {}
        ro.close()
        torch.cuda.synchronize()

    for i in range(8):
        cycle(i)
    free = [torch.cuda.mem_get_info()[0]]
    for i in range(40):
        cycle(i)
        free.append(torch.cuda.mem_get_info()[0])
    print(dict(free_mb=[round(f / 2**20, 1) for f in free[::8]]))
    assert free[-1] >= free[0] - (2 << 20), (free[0], free[-1])
