"""GPU parity of the uneven-batch plan (pairs with different n and k) against the FP64 oracle.

Every pair's C, info, A, B and, after the backward replay, dF_x and dF_y are
compared with the oracle run on that pair alone: relative Frobenius error
<= 1e-5 (float32 arrays), info bit-exact.  Graph replays are repeated with
inputs rewritten in place and unrelated eager work in between; every replay is
checked.
"""
import numpy as np
import pytest

import oracle
from paper_2604_10377_amd import synth
from tests.conftest import rel_fro

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def F(dev):
    from paper_2604_10377_amd import fmap
    return fmap


def _device_pairs(pairs, dev):
    import torch
    out = []
    for p in pairs:
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
        out.append(dict(phi_x=t(p.phi_x), phi_y=t(p.phi_y), mass_x=t(p.mass_x), mass_y=t(p.mass_y),
                        feat_x=t(p.feat_x), feat_y=t(p.feat_y), evals_x=t(p.evals_x), evals_y=t(p.evals_y),
                        lam=t(np.asarray([p.lam]))))
    return out


def _oracle(p, mask, gamma, feat_x=None, feat_y=None):
    fx = p.feat_x if feat_x is None else feat_x
    fy = p.feat_y if feat_y is None else feat_y
    A, B, D, C, info = oracle.forward_pair(p.phi_x, p.mass_x, fx, p.phi_y, p.mass_y, fy, p.evals_x, p.evals_y,
                                           p.lam, mask, gamma)
    dA, dB, _ = oracle.solve_backward(A, B, C, D, p.lam, p.dC)
    return dict(A=A, B=B, C=C, info=info, dFx=oracle.project_backward(p.phi_x, p.mass_x, dA),
                dFy=oracle.project_backward(p.phi_y, p.mass_y, dB))


def _check(plan, pairs, refs, with_bwd=True, with_AB=False):
    for i, (p, r) in enumerate(zip(pairs, refs)):
        tag = f"pair {i} (n_x={p.n_x}, n_y={p.n_y}, k={p.k})"
        assert rel_fro(plan.C[i].cpu().numpy(), r["C"]) <= TOL, tag
        assert np.array_equal(plan.info[i].cpu().numpy(), r["info"]), tag
        if with_AB:
            assert rel_fro(plan.A[i].cpu().numpy(), r["A"]) <= TOL, tag
            assert rel_fro(plan.B[i].cpu().numpy(), r["B"]) <= TOL, tag
        if with_bwd:
            assert rel_fro(plan.dF_x[i].cpu().numpy(), r["dFx"]) <= TOL, tag
            assert rel_fro(plan.dF_y[i].cpu().numpy(), r["dFy"]) <= TOL, tag


# k values cover both row-solve kernels (<= 64 in registers, > 64 tiled); n is ragged;
# d = 200 leaves a partial 256-column block
RAGGED = dict(pairs=7, d=200, n_lo=300, n_hi=3100, ks=(17, 30, 64, 80))


@pytest.mark.parametrize("mask,recompute", [(synth.MASK_LAPLACIAN, False), (synth.MASK_RESOLVENT, True)])
def test_plan_ragged_forward_backward(F, dev, mask, recompute):
    import torch
    pairs = synth.workload_ragged(**RAGGED)
    assert len({p.k for p in pairs}) >= 3
    print("plan ragged:", [(p.n_x, p.n_y, p.k) for p in pairs], "mask", mask, "recompute", recompute, flush=True)
    dpairs = _device_pairs(pairs, dev)
    plan = F.FmapPlan(dpairs, mask, 0.5, backward=True, recompute=recompute, want_AB=True)
    for i, p in enumerate(pairs):
        plan.dC[i].copy_(torch.from_numpy(p.dC))
    plan.forward()
    plan.backward()
    torch.cuda.synchronize()
    _check(plan, pairs, [_oracle(p, mask, 0.5) for p in pairs], with_AB=True)
    plan.close()


# more k groups than solve branches: six groups, so that two register-solve groups share one side stream in
# the forward (the tiled k = 70 and 100 groups stay on the capturing stream) and the backward's groups wrap
# round the four streams.  d = 128 exceeds every k: with d < k, A A^T is singular and the row systems are
# conditioned by lambda alone (about 1.7e3 here at d = 64), beyond what the float32 tolerance allows
MANY_GROUPS = dict(pairs=8, d=128, n_lo=200, n_hi=900, ks=(8, 17, 30, 50, 70, 100))


def test_plan_more_groups_than_branches(F, dev):
    import torch
    pairs = synth.workload_ragged(**MANY_GROUPS)
    assert {p.k for p in pairs} == set(MANY_GROUPS["ks"])
    print("plan six groups:", [(p.n_x, p.n_y, p.k) for p in pairs], flush=True)
    dpairs = _device_pairs(pairs, dev)
    plan = F.FmapPlan(dpairs, synth.MASK_LAPLACIAN, 0.5, backward=True, want_AB=True)
    for i, p in enumerate(pairs):
        plan.dC[i].copy_(torch.from_numpy(p.dC))
    refs = [_oracle(p, synth.MASK_LAPLACIAN, 0.5) for p in pairs]
    for _ in range(2):  # two replays of each graph, checked after the second
        plan.forward()
        plan.backward()
        torch.cuda.synchronize()
    _check(plan, pairs, refs, with_AB=True)
    plan.close()


# the large-k groups of the uneven workload: k = 120 (four K steps of 32 in the backward projection items)
# and k = 150 (five), beside a register-solve group; n spans several vertex tiles with ragged tails
LARGE_GROUPS = dict(pairs=6, d=256, n_lo=900, n_hi=4100, ks=(50, 120, 150))


@pytest.mark.parametrize("recompute", [False, True])
def test_plan_large_k_groups(F, dev, recompute):
    import torch
    pairs = synth.workload_ragged(**LARGE_GROUPS)
    assert {p.k for p in pairs} >= {120, 150}
    print("plan large-k groups:", [(p.n_x, p.n_y, p.k) for p in pairs], "recompute", recompute, flush=True)
    dpairs = _device_pairs(pairs, dev)
    plan = F.FmapPlan(dpairs, synth.MASK_LAPLACIAN, 0.5, backward=True, recompute=recompute, want_AB=True)
    for i, p in enumerate(pairs):
        plan.dC[i].copy_(torch.from_numpy(p.dC))
    plan.forward()
    plan.backward()
    torch.cuda.synchronize()
    _check(plan, pairs, [_oracle(p, synth.MASK_LAPLACIAN, 0.5) for p in pairs], with_AB=True)
    plan.close()


def test_plan_ragged_workload_full_size(F, dev):
    """The uneven workload at full size: 64 pairs, n ~ U{2000..20000} per shape, k in {30, 50, 80, 120},
    d = 256, Laplacian mask, lambda per pair; one captured forward and backward.  Checked against the
    oracle: the first pair of every k group and the pair with the most vertices."""
    import torch
    pairs = synth.workload_ragged()
    dpairs = _device_pairs(pairs, dev)
    plan = F.FmapPlan(dpairs, synth.MASK_LAPLACIAN, 0.5, backward=True, want_AB=True)
    for i, p in enumerate(pairs):
        plan.dC[i].copy_(torch.from_numpy(p.dC))
    plan.forward()
    plan.backward()
    torch.cuda.synchronize()
    pick = sorted({next(i for i, p in enumerate(pairs) if p.k == k) for k in {p.k for p in pairs}} |
                  {max(range(len(pairs)), key=lambda i: pairs[i].n_x + pairs[i].n_y)})
    print("plan full-size ragged: checking pairs", [(i, pairs[i].n_x, pairs[i].n_y, pairs[i].k) for i in pick],
          flush=True)
    sel = [pairs[i] for i in pick]

    class View:  # the checked pairs' slots of the plan
        C = [plan.C[i] for i in pick]
        info = [plan.info[i] for i in pick]
        A = [plan.A[i] for i in pick]
        B = [plan.B[i] for i in pick]
        dF_x = [plan.dF_x[i] for i in pick]
        dF_y = [plan.dF_y[i] for i in pick]

    _check(View, sel, [_oracle(p, synth.MASK_LAPLACIAN, 0.5) for p in sel], with_AB=True)
    plan.close()


# shapes of a few stages plus a tail (k = 68: sliced forward and the large-k backward), and shapes below
# one stage (n < 32: the general kernels only)
SMALL = [dict(pairs=5, d=256, n_lo=70, n_hi=140, ks=(8, 30, 68)), dict(pairs=3, d=64, n_lo=10, n_hi=31, ks=(8,))]


@pytest.mark.parametrize("cfg", SMALL, ids=["stages+tails", "below-one-stage"])
def test_plan_small_shapes(F, dev, cfg):
    import torch
    pairs = synth.workload_ragged(**cfg)
    print("plan small:", [(p.n_x, p.n_y, p.k) for p in pairs], flush=True)
    dpairs = _device_pairs(pairs, dev)
    plan = F.FmapPlan(dpairs, synth.MASK_LAPLACIAN, 0.5, backward=True, want_AB=True)
    for i, p in enumerate(pairs):
        plan.dC[i].copy_(torch.from_numpy(p.dC))
    plan.forward()
    plan.backward()
    torch.cuda.synchronize()
    _check(plan, pairs, [_oracle(p, synth.MASK_LAPLACIAN, 0.5) for p in pairs], with_AB=True)
    plan.close()


def test_plan_replays_follow_inputs(F, dev):
    """Three replays; between them the features are rewritten in place and eager work runs."""
    import torch
    pairs = synth.workload_ragged(pairs=4, d=128, n_lo=500, n_hi=2000, ks=(30, 50))
    dpairs = _device_pairs(pairs, dev)
    plan = F.FmapPlan(dpairs, synth.MASK_LAPLACIAN, 0.5, backward=True)
    for i, p in enumerate(pairs):
        plan.dC[i].copy_(torch.from_numpy(p.dC))
    rng = np.random.default_rng(5)
    for rep in range(3):
        print("replay", rep, flush=True)
        fx = [(p.feat_x * (1.0 + 0.5 * rep) + 0.1 * rng.standard_normal(p.feat_x.shape)).astype(np.float32)
              for p in pairs]
        fy = [(p.feat_y + 0.1 * rng.standard_normal(p.feat_y.shape)).astype(np.float32) for p in pairs]
        for i in range(len(pairs)):
            dpairs[i]["feat_x"].copy_(torch.from_numpy(fx[i]))
            dpairs[i]["feat_y"].copy_(torch.from_numpy(fy[i]))
        x = torch.randn(512, 512, device=dev)
        (x @ x).sum().item()  # unrelated eager work and a synchronisation between replays
        plan.forward()
        plan.backward()
        torch.cuda.synchronize()
        _check(plan, pairs, [_oracle(p, synth.MASK_LAPLACIAN, 0.5, fx[i], fy[i]) for i, p in enumerate(pairs)])
    plan.close()


def test_plan_tuning_cache_round_trip(F, dev, tmp_path):
    """A second plan on the same workload takes the tuned parameters from the cache and gives identical C."""
    import torch
    pairs = synth.workload_ragged(pairs=3, d=64, n_lo=200, n_hi=900, ks=(20, 40))
    dpairs = _device_pairs(pairs, dev)
    cache = tmp_path / "tune.txt"
    p1 = F.FmapPlan(dpairs, synth.MASK_RESOLVENT, 0.5, backward=False, tune_cache=cache)
    t1 = p1.tuning()
    assert not t1["from_cache"]
    assert t1["chunk"] in (512, 1024, 2048) and t1["systems_per_wg"] in (1, 2, 4) and t1["grid"] >= 1
    assert cache.read_text().count("\n") == 1
    p2 = F.FmapPlan(dpairs, synth.MASK_RESOLVENT, 0.5, backward=False, tune_cache=cache)
    t2 = p2.tuning()
    assert t2["from_cache"] and {k: t2[k] for k in ("chunk", "grid", "systems_per_wg")} == \
        {k: t1[k] for k in ("chunk", "grid", "systems_per_wg")}
    g1, g2 = p1.groups(), p2.groups()
    assert [g["k"] for g in g1] == [20, 40] and g1 == g2
    assert all(g["systems_per_wg"] in (1, 2, 4) for g in g1)
    # a plan with a backward pass has its own cache entry (the backward parameters are tuned for it)
    p3 = F.FmapPlan(dpairs, synth.MASK_RESOLVENT, 0.5, backward=True, tune_cache=cache)
    assert not p3.tuning()["from_cache"]
    assert cache.read_text().count("\n") == 2
    p3.close()
    p1.forward()
    p2.forward()
    torch.cuda.synchronize()
    for i, p in enumerate(pairs):
        assert torch.equal(p1.C[i], p2.C[i])
        assert rel_fro(p1.C[i].cpu().numpy(), _oracle(p, synth.MASK_RESOLVENT, 0.5)["C"]) <= TOL
    with pytest.raises(F.FmapError):
        p1.backward()  # created without backward slots
    p1.close()
    p2.close()


def test_plan_single_pair_matches_batched_entry_points(F, dev):
    """A one-pair plan gives the same C as fmap_project + fmap_solve (same kernels, same order)."""
    import torch
    b = synth.make_batch("t", 91, 1, 2345, 50, 256, mask=synth.MASK_RESOLVENT)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    dp = [dict(phi_x=t(b.phi[0]), phi_y=t(b.phi[1]), mass_x=t(b.mass[0]), mass_y=t(b.mass[1]), feat_x=t(b.feat[0]),
               feat_y=t(b.feat[1]), evals_x=t(b.evals[0]), evals_y=t(b.evals[1]), lam=t(b.lam[:1]))]
    plan = F.FmapPlan(dp, synth.MASK_RESOLVENT, 0.5, backward=False)
    plan.forward()
    AB = F.fmap_project(t(b.phi), t(b.mass), t(b.feat))
    C, _, info, _ = F.fmap_solve(AB[:1], AB[1:], t(b.evals[:1]), t(b.evals[1:]), t(b.lam), synth.MASK_RESOLVENT, 0.5)
    torch.cuda.synchronize()
    assert rel_fro(plan.C[0].cpu().numpy(), C[0].cpu().numpy()) <= 1e-6
    assert torch.equal(plan.info[0], info[0])
    plan.close()
