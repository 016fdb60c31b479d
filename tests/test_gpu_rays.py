"""GPU parity of the secondary-ray queries (msp_bvh_build,
msp_trace_transmittance, msp_trace_closest) against the brute-force ray
oracle through the C ABI, and the hierarchy's structure checked on the host.

Rays whose oracle test puts a face within a float32 decision margin (an edge
or an interval end) may see that face or not: their transmittance must equal
the oracle's product for some choice of those faces, and their closest hit is
compared only when no such face is nearer than the oracle's hit."""
import itertools

import numpy as np
import pytest

from oracle import convert as oc
from oracle import rays as ory
from paper_2502_07754_amd import scenes
from tests.helpers import faces_f32, to_gpu

pytestmark = pytest.mark.gpu

T_TOL = 2e-5


def _say(*a):
    print(*a, flush=True)


def _fans(n, seed, K=8, lo=0.02, hi=0.2, flat=True):
    g = scenes.gaussians(n, seed, lo, hi, flat=flat)
    return faces_f32(oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, K, 2.0))


def _rays(n, seed, spread=1.3, tmax=np.inf):
    rng = np.random.default_rng(seed)
    O = rng.uniform(-spread, spread, (3, n)).astype(np.float32)
    D = rng.normal(size=(3, n)).astype(np.float32)
    t0 = np.full(n, 1e-4, np.float32)
    t1 = np.full(n, tmax, np.float32)
    return O, D, t0, t1


def _gpu_rays(O, D, t0, t1):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (O, D, t0, t1)]


def _check_transmittance(f, O, D, t0, t1, T):
    f64 = {k: v.astype(np.float64) if v.dtype == np.float32 else v for k, v in f.items()}
    ref = ory.transmittance(f64, O, D, t0, t1)
    flags = ory.near_boundary(f64, O, D, t0, t1)
    n_flag = 0
    for r in range(O.shape[1]):
        if abs(T[r] - ref[r]) <= T_TOL:
            continue
        fl = flags[r]
        assert 0 < len(fl) <= 6, (r, T[r], ref[r], len(fl))
        n_flag += 1
        t, u, v, hit = ory.intersect(f64["pos"], f64["idx"], O[:, r], D[:, r])
        a = ory.hit_alpha(f64["opacity"], f64["idx"], u, v)
        sel = hit & (t > t0[r]) & (t < t1[r])
        base_sel = sel.copy()
        base_sel[fl] = False
        base = np.prod(1 - a[base_sel])
        ok = any(abs(T[r] - base * np.prod(1 - a[list(S)])) <= T_TOL
                 for m in range(len(fl) + 1) for S in itertools.combinations(fl, m))
        assert ok, (r, T[r], ref[r])
    return ref, n_flag


@pytest.mark.parametrize("n_gauss,seed", [(1, 1), (3, 2), (300, 3), (2000, 4)])
def test_bvh_structure(gpu, n_gauss, seed):
    f = _fans(n_gauss, seed)
    F = f["idx"].shape[1]
    _say("bvh structure", F)
    b = gpu.Bvh(to_gpu(f))
    nodes, leaves, box = [x.cpu().numpy() for x in b.export()]
    st = b.status()
    assert st["n_leaves"] == F and not st["overflowed"]
    fid = leaves[:, 12].view(np.int32)
    assert np.array_equal(np.sort(fid), np.arange(F))
    P, I, op = f["pos"], f["idx"], f["opacity"]
    p0 = P[:, I[0, fid]].T
    assert np.array_equal(leaves[:, 0:3], p0)
    assert np.array_equal(leaves[:, 4:7], (P[:, I[1, fid]].T - p0).astype(np.float32))
    assert np.array_equal(leaves[:, 8:11], (P[:, I[2, fid]].T - p0).astype(np.float32))
    assert np.array_equal(leaves[:, [3, 7, 11]], np.stack([op[I[k, fid]] for k in range(3)], 1))

    def leaf_box(j):
        q = np.stack([leaves[j, 0:3], leaves[j, 0:3] + leaves[j, 4:7], leaves[j, 0:3] + leaves[j, 8:11]])
        return q.min(0), q.max(0)

    seen = []

    def walk(c, depth):
        """box of the subtree; checks that each stored child box holds its subtree"""
        assert depth <= 64
        if c < 0:
            seen.append(~c)
            return leaf_box(~c)
        nd = nodes[c]
        kids = nd[12:14].view(np.int32)
        out_lo, out_hi = np.full(3, np.inf), np.full(3, -np.inf)
        for s, k in enumerate(kids):
            lo, hi = walk(int(k), depth + 1)
            assert np.all(nd[6 * s:6 * s + 3] <= lo) and np.all(nd[6 * s + 3:6 * s + 6] >= hi)
            out_lo, out_hi = np.minimum(out_lo, lo), np.maximum(out_hi, hi)
        return out_lo, out_hi

    lo, hi = walk(0 if F > 1 else ~0, 0)
    assert sorted(seen) == list(range(F))
    assert np.all(box[:3] <= lo) and np.all(box[3:] >= hi)


@pytest.mark.parametrize("n_gauss,seed,tmax", [(2000, 5, np.inf), (500, 6, 1.5), (1, 7, np.inf)])
def test_transmittance_parity(gpu, n_gauss, seed, tmax):
    f = _fans(n_gauss, seed, lo=0.05, hi=0.3)
    O, D, t0, t1 = _rays(3000 if n_gauss > 1 else 500, seed, tmax=tmax)
    if n_gauss == 1:
        # aim every ray at the single fan's centre from a random origin
        c = f["pos"][:, 0:1].astype(np.float64)
        D = (c - O.astype(np.float64) + np.random.default_rng(1).normal(0, 0.1, O.shape)).astype(np.float32)
    _say("transmittance", n_gauss, tmax)
    b = gpu.Bvh(to_gpu(f))
    T = b.transmittance(*_gpu_rays(O, D, t0, t1)).cpu().numpy().astype(np.float64)
    ref, n_flag = _check_transmittance(f, O, D, t0, t1, T)
    _say("  rays", len(T), "occluded", int(np.sum(ref < 1)), "flagged", n_flag)
    assert np.sum(ref < 1) > 0.2 * len(T)
    assert n_flag <= 0.02 * len(T)
    assert not b.status()["overflowed"]


@pytest.mark.parametrize("alpha_min", [0.0, 0.3])
def test_closest_parity(gpu, alpha_min):
    f = _fans(2000, 8, lo=0.05, hi=0.3)
    O, D, t0, t1 = _rays(3000, 9)
    b = gpu.Bvh(to_gpu(f))
    t, fid, u, v = [x.cpu().numpy() for x in b.closest(*_gpu_rays(O, D, t0, t1), alpha_min=alpha_min)]
    f64 = {k: x.astype(np.float64) if x.dtype == np.float32 else x for k, x in f.items()}
    rt, rf, ru, rv = ory.closest_hit(f64, O, D, t0, t1, alpha_min)
    flags = ory.near_boundary(f64, O, D, t0, t1)
    compared = 0
    for r in range(O.shape[1]):
        fl = flags[r]
        # a face near a decision margin and not farther than the oracle's hit may change the answer
        if len(fl):
            tt, uu, vv, _ = ory.intersect(f64["pos"], f64["idx"], O[:, r], D[:, r])
            if np.any(tt[fl] <= (rt[r] if rf[r] >= 0 else np.inf) * (1 + 1e-5) + 1e-6):
                continue
        # two hits within float32 resolution of each other may come in either order
        if rf[r] >= 0:
            tt, uu, vv, hh = ory.intersect(f64["pos"], f64["idx"], O[:, r], D[:, r])
            a = ory.hit_alpha(f64["opacity"], f64["idx"], uu, vv)
            near = hh & (tt > t0[r]) & (tt < t1[r]) & (a >= alpha_min) & (np.abs(tt - rt[r]) <= 1e-5 * abs(rt[r]))
            if near.sum() > 1:
                continue
        compared += 1
        assert fid[r] == rf[r], (r, fid[r], rf[r], t[r], rt[r])
        if rf[r] >= 0:
            assert abs(t[r] - rt[r]) <= 1e-5 * max(1.0, abs(rt[r]))
            assert abs(u[r] - ru[r]) <= 1e-4 and abs(v[r] - rv[r]) <= 1e-4
        else:
            assert np.isinf(t[r])
    _say("closest", alpha_min, "compared", compared, "hits", int(np.sum(rf >= 0)))
    assert compared >= 0.98 * O.shape[1] and np.sum(rf >= 0) > 0.2 * O.shape[1]


def test_rays_edge_cases(gpu):
    import torch
    O, D, t0, t1 = _rays(100, 10)
    empty = dict(pos=np.zeros((3, 0), np.float32), opacity=np.zeros(0, np.float32), rgb=np.zeros((3, 0), np.float32),
                 idx=np.zeros((3, 0), np.int32))
    b = gpu.Bvh(to_gpu(empty))
    assert np.all(b.transmittance(*_gpu_rays(O, D, t0, t1)).cpu().numpy() == 1.0)
    t, fid, _, _ = b.closest(*_gpu_rays(O, D, t0, t1))
    assert np.all(fid.cpu().numpy() == -1) and np.all(np.isinf(t.cpu().numpy()))
    # no rays at all
    f = _fans(50, 11)
    b = gpu.Bvh(to_gpu(f))
    z = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    e = torch.zeros((0,), dtype=torch.float32, device="cuda")
    assert b.transmittance(z, z, e, e).numel() == 0
    # an empty interval sees nothing
    T = b.transmittance(*_gpu_rays(O, D, np.full(100, 2.0, np.float32), np.full(100, 1.0, np.float32)))
    assert np.all(T.cpu().numpy() == 1.0)
    # identical fans stacked on one place: equal Morton codes, equal t; the smaller face id wins
    g = _fans(1, 12)
    V1, F1, reps = g["pos"].shape[1], g["idx"].shape[1], 64
    rep = dict(pos=np.tile(g["pos"], (1, reps)), opacity=np.tile(g["opacity"], reps), rgb=np.tile(g["rgb"], (1, reps)),
               idx=np.concatenate([g["idx"] + V1 * k for k in range(reps)], axis=1).astype(np.int32))
    b = gpu.Bvh(to_gpu(rep))
    c = g["pos"][:, 0:1]
    O2 = (c + np.array([[0.0], [0.0], [2.0]])).astype(np.float32).repeat(8, axis=1)
    D2 = np.tile(np.array([[0.001], [0.002], [-1.0]], np.float32), (1, 8))
    t, fid, _, _ = b.closest(*_gpu_rays(O2, D2, np.zeros(8, np.float32), np.full(8, np.inf, np.float32)))
    fid = fid.cpu().numpy()
    assert np.all(fid >= 0) and np.all(fid < F1)
    assert not b.status()["overflowed"]


def test_transmittance_full_size_sampled(gpu):
    """The shadow-ray workload's scene (500k flat Gaussians, K = 16: 8M faces)
    and its rays; 12 sampled rays against the oracle, the rest by the product's
    bounds (0 <= T <= 1)."""
    g = scenes.gaussians(500_000, 0, 0.01, 0.1, flat=True)
    f = faces_f32(oc.convert_fan(g.mean, g.scale, g.quat, g.opacity, g.rgb, 16, 2.0))
    b = gpu.Bvh(to_gpu(f))
    O, D, t0, t1 = scenes.shadow_rays(1_000_000, 0)
    T = b.transmittance(*_gpu_rays(O, D, t0, t1)).cpu().numpy().astype(np.float64)
    assert np.all((T >= 0) & (T <= 1)) and not b.status()["overflowed"]
    sample = np.random.default_rng(5).choice(len(T), 12, replace=False)
    ref, n_flag = _check_transmittance(f, O[:, sample], D[:, sample], t0[sample], t1[sample], T[sample])
    _say("full size: occluded", float(np.mean(T < 1)), "sampled", ref, "flagged", n_flag)
    assert n_flag <= 1


def test_ray_order_gives_the_same_results(gpu):
    """Tracing in any order (a random permutation, the Morton order of the
    origins) gives bit-identical results at each ray's own index; order
    entries outside [0, n) are skipped."""
    import torch
    f = _fans(500, 13, lo=0.05, hi=0.3)
    O, D, t0, t1 = _rays(4000, 14)
    b = gpu.Bvh(to_gpu(f))
    rays = _gpu_rays(O, D, t0, t1)
    T = b.transmittance(*rays).cpu().numpy()
    hit = [x.cpu().numpy() for x in b.closest(*rays, alpha_min=0.2)]
    perm = torch.from_numpy(np.random.default_rng(3).permutation(4000).astype(np.int32)).cuda()
    for order in (perm, gpu.point_order(rays[0])):
        assert np.array_equal(np.sort(order.cpu().numpy()), np.arange(4000))
        assert np.array_equal(b.transmittance(*rays, order=order).cpu().numpy(), T)
        got = [x.cpu().numpy() for x in b.closest(*rays, alpha_min=0.2, order=order)]
        for a, c in zip(got, hit):
            assert np.array_equal(a, c)
    bad = np.arange(4000, dtype=np.int32)
    bad[:10] = 4000
    bad[10:20] = -1
    T2 = b.transmittance(*rays, order=torch.from_numpy(bad).cuda())
    assert np.array_equal(T2.cpu().numpy()[20:], T[20:])
