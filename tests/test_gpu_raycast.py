"""Raycast contact-depth backend (include/tg_raycast.h) against the FP64 brute-force oracle,
through the C ABI.

The GPU places the probe in the object frame in FP32 (about 1e-8 m off the FP64 position) and
runs the closest-point and ray tests in FP32 on a BVH; the oracle visits every triangle in FP64.
The depth is unique: |d_gpu - d_ref| <= 5e-7 m (FP32 positions, a few roundings in the
closest-point and ray arithmetic, ten times over).  The winning triangle is not unique where two
triangles tie (a probe closest to a shared edge or vertex, a ray through an edge), so it is
checked for validity: the oracle's penetration of the GPU's triangle alone is within the same
bar of the depth, and the GPU normal equals the oracle's normal where the two pick the same
triangle (1e-5).

Against the analytic SDF on the tessellated sphere: outside the object the raycast depth is
R - (distance to the mesh), within the mesh's sagitta of R - phi; inside it is R + (the axial
distance to the surface), never below R - phi - sagitta.
"""
import numpy as np
import pytest

import oracle
from paper_2606_22332_amd import synth

pytestmark = pytest.mark.gpu
TOL = 5e-7


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_gpu(torch, sc, inp, meshes):
    from paper_2606_22332_amd import binding as B
    rc = B.Raycast(sc, meshes)
    d = B.to_device(inp)
    dep, nm, tri = rc.rollout(d)
    torch.cuda.synchronize()
    rc.close()
    return dep.cpu().numpy(), nm.cpu().numpy(), tri.cpu().numpy()


def run_oracle(sc, inp, meshes, tri_query=None):
    lay = sc.layout
    return oracle.raycast_run(lay.link_offset, lay.pos, lay.normal, lay.radius, meshes, inp.link_state, inp.obj_id,
                              inp.obj_state, tri_query=tri_query)


def check(g, ref, sc, inp, meshes):
    gd, gn, gt = g
    rd, rn, rt, tp = ref
    err = np.abs(gd - rd)
    info = dict(max_depth_err_um=float(err.max() * 1e6), contacts=float((rd > TOL).mean()),
                same_triangle=float(np.mean(gt[rd > TOL] == rt[rd > TOL])) if (rd > TOL).any() else 1.0)
    assert np.all(err <= TOL), info
    c = rd > TOL
    assert np.all(gt[c] >= 0), info
    assert np.all(tp[c] >= rd[c] - TOL), info                        # the GPU's triangle is as deep
    same = c & (gt == rt)
    nerr = np.abs(gn - rn).max(axis=1)
    assert np.all(nerr[same] <= 1e-5), info
    ln = np.linalg.norm(gn, axis=1)
    assert np.all(np.abs(ln[c] - 1) <= 1e-5), info
    return info


@pytest.mark.parametrize("moving", [False, True])
def test_hand_parity(torch_cuda, moving):
    sc = synth.make_scene("c2", num_envs=24, num_steps=4)
    inp = synth.make_inputs(sc)
    if moving:
        inp.obj_state = synth.random_object_state(sc, 4)
    oid = inp.obj_id.copy()
    oid[:, 3] = -1
    oid[:, 7] = 50
    inp.obj_id = oid
    meshes = synth.object_meshes(sc.grids)
    g = run_gpu(torch_cuda, sc, inp, meshes)
    ref = run_oracle(sc, inp, meshes, tri_query=g[2])
    info = check(g, ref, sc, inp, meshes)
    print(dict(moving=moving, **info))
    assert info["contacts"] > 0.05
    assert np.all(g[0][:, [3, 7]] == 0) and np.all(g[2][:, [3, 7]] == -1)


def test_against_the_analytic_sphere(torch_cuda):
    sc = synth.make_scene("c2", num_envs=64, num_steps=3)
    inp = synth.make_inputs(sc)
    inp.obj_id = np.zeros_like(inp.obj_id)                    # object 0 is the sphere
    s = sc.grids[0].shape
    assert s["family"] == "sphere"
    meshes = synth.object_meshes(sc.grids, detail=4)
    v, t = meshes[0]
    vv = v.astype(float)
    cen = vv[t].mean(axis=1)
    nrm = np.cross(vv[t[:, 1]] - vv[t[:, 0]], vv[t[:, 2]] - vv[t[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    sag = s["r"] - np.min(np.sum(cen * nrm, axis=1))
    gd, gn, gt = run_gpu(torch_cuda, sc, inp, meshes)
    # probe centres in the object frame (objects static at the origin)
    lay = sc.layout
    L, E = lay.num_links, sc.num_envs
    link_of = np.repeat(np.arange(L), np.diff(lay.link_offset))
    ls = inp.link_state.astype(np.float64)
    S = ls.shape[0]
    q = np.zeros((S, E, lay.num_taxels, 3))
    for si in range(S):
        for e in range(E):
            for l in range(L):
                c = ls[si, :, e * L + l]
                w, x, y, z = c[3:7]
                Rm = np.array([[1-2*(y*y+z*z), 2*(x*y-w*z), 2*(x*z+w*y)], [2*(x*y+w*z), 1-2*(x*x+z*z), 2*(y*z-w*x)],
                               [2*(x*z-w*y), 2*(y*z+w*x), 1-2*(x*x+y*y)]])
                js = np.nonzero(link_of == l)[0]
                q[si, e, js] = c[:3] + lay.pos[js].astype(float) @ Rm.T
    phi = np.linalg.norm(q, axis=-1) - s["r"]
    R = lay.radius.astype(float)[None, None, :]
    dsdf = np.maximum(R - phi, 0)
    outside = (phi > 0) & (dsdf > 0)
    inside = phi < 0
    assert outside.any() and inside.any()
    assert np.all(np.abs(gd[outside] - dsdf[outside]) <= sag + TOL)
    assert np.all(gd[inside] >= dsdf[inside] - sag - TOL)
    print(dict(sagitta_um=sag * 1e6, outside=int(outside.sum()), inside=int(inside.sum()),
               outside_max_um=float(np.abs(gd[outside] - dsdf[outside]).max() * 1e6)))


def test_full_size_sampled(torch_cuda):
    """The benchmark's launch (4096 envs x 200 taxels x 100 steps) checked on sampled envs."""
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    sc = synth.make_scene("c2")
    inp = synth.make_inputs(sc)
    meshes = synth.object_meshes(sc.grids)
    rc = B.Raycast(sc, meshes)
    dep, nm, tri = rc.rollout(B.to_device(inp))
    envs = np.array([0, 1, 2048, 4095])
    idx = torch.as_tensor(envs, device="cuda")
    g = (dep[:, idx].cpu().numpy(), nm[:, :, idx].cpu().numpy(), tri[:, idx].cpu().numpy())
    torch.cuda.synchronize()
    rc.close()
    sub = synth.subset_envs(inp, envs, sc.layout.num_links)
    sc_sub = synth.make_scene("c2", num_envs=len(envs))
    ref = run_oracle(sc_sub, sub, meshes, tri_query=g[2])
    print(check(g, ref, sc_sub, sub, meshes))


def test_rejects_bad_meshes(torch_cuda):
    from paper_2606_22332_amd import binding as B
    sc = synth.make_scene("c2", num_envs=2, num_steps=1)
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float32) * 0.01
    with pytest.raises(B.TgError):
        B.Raycast(sc, [(v, np.array([[0, 1, 1]], np.int32))])            # degenerate
    with pytest.raises(B.TgError):
        B.Raycast(sc, [(v, np.array([[0, 1, 7]], np.int32))])            # index out of range
    bad = v.copy(); bad[2, 1] = np.nan
    with pytest.raises(B.TgError):
        B.Raycast(sc, [(bad, np.array([[0, 1, 2]], np.int32))])
