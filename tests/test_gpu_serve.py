"""The request loop: continuous batching, memory-budgeted admission and
resident meshes.  Every served output must equal the same request computed
on a context of its own (a fresh selection, or a warm start from the mesh's
previous support set when the server kept it), within 1e-12 max|d|."""
import numpy as np
import pytest
import torch

import synth
import paper_2004_04817_amd as gcb
from paper_2004_04817_amd import serving

pytestmark = pytest.mark.gpu

TOL_SAME = 1e-12


def alone_reference(served):
    """Recompute every request in its admission order on private contexts."""
    refs = {}        # mesh key -> context holding the mesh's kept support set
    outs = {}
    order = sorted(served, key=lambda s: s.result["t_admit"])
    extra = []
    for s in order:
        r = s.result
        if r["warm"]:
            c = refs[s.req.key]
            c.set_displacement(s.disp)
            c.set_params(s.radius, s.m, s.tol_abs, seed=s.seed, warm_start=True)
        else:
            c = gcb.Context(0)
            c.set_boundary(s.xyz, s.disp)
            c.set_params(s.radius, s.m, s.tol_abs, seed=s.seed)
            if r["kept"]:
                refs[s.req.key] = c
            else:
                extra.append(c)
        info = c.select()
        assert info["nc"] == r["nc"] and info["iterations"] == r["iterations"], s.req
        outs[s.ticket] = c.deform(s.vol)
    torch.cuda.synchronize()
    for c in list(refs.values()) + extra:
        c.close()
    return outs


def check_same(served):
    ref = alone_reference(served)
    for s in served:
        assert s.result["state"] == 3, (s.req, s.result["state"])
        md = float(np.sqrt((s.disp ** 2).sum(axis=1)).max())
        d = (s.out - ref[s.ticket]).abs().max().item() if s.out.numel() else 0.0
        assert d <= TOL_SAME * md, (s.req, d)


def small_stream(n, repeat_p, scale=0.08):
    return serving.materialise(synth.config_requests(n, rate=200.0, repeat_p=repeat_p, size_scale=scale))


def test_served_mix_equals_alone():
    items = small_stream(14, 0.4)
    pool = serving.volume_pool(40_000, "cuda")
    with gcb.Server(0, hbm_budget=4 << 30, max_active=8) as srv:
        served = serving.replay(srv, items, pool, nv_per_nb=6, iterations=8)
        assert any(s.result["warm"] for s in served)
        # requests overlapped: some were admitted before an earlier one finished
        adm = sorted((s.result["t_admit"], s.result["t_done"]) for s in served)
        assert any(adm[i + 1][0] < adm[i][1] for i in range(len(adm) - 1))
        check_same(served)


TAU_REL = 1e-9      # near-tie tolerance of the follow-mode replay, relative to max|d|
TOL_ORACLE = 1e-9   # Eq. 6 outputs against the oracle's, relative to max|d|


def check_against_oracle(served, n_points=2000):
    """Every served request against the FP64 oracle (Algorithm 1 + Eq. 6 per request).

    Fresh requests: the recorded support sequence equals oracle.select's, or the
    oracle's follow-mode replay certifies every iteration of the served run.
    Warm starts: the same against the oracle's warm start from the support set
    the mesh kept (the served sequence of the previous request of that key).
    Outputs: sampled Eq. 6 displacements against oracle.interpolate with the
    oracle's weights for the served support set."""
    import oracle
    kept = {}
    rng = np.random.default_rng(7)
    stats = {"same": 0, "certified": 0, "warm": 0}
    for s in sorted(served, key=lambda s: s.result["t_admit"]):
        r = s.result
        assert r["state"] == 3 and "support" in r, (s.req, r["state"])
        S = r["support"]
        lg = r["log"]
        md = float(np.sqrt((s.disp ** 2).sum(axis=1)).max())
        warm_S = kept[s.req.key] if r["warm"] else None
        o = oracle.select(s.xyz, s.disp, s.radius, s.m, s.tol_abs, seed=s.seed, warm_S=warm_S)
        assert r["iterations"] == len(lg["log_group"])
        if len(o.S) == len(S) and np.array_equal(o.S, S):
            stats["same"] += 1
            assert o.iterations == r["iterations"], s.req
            W = o.W
        else:
            bad, reason, _ = oracle.validate(s.xyz, s.disp, s.radius, s.m, s.tol_abs, S, lg["log_group"],
                                             lg["log_node"], lg["log_appended"], TAU_REL * md, seed=s.seed,
                                             warm_S=warm_S)
            assert bad == -1, (s.req, bad, reason)
            stats["certified"] += 1
            W = oracle.solve_on_support(s.xyz, S, s.radius, s.disp)
        stats["warm"] += int(bool(r["warm"]))
        # the served weights are the oracle's solve on the same support set
        assert np.abs(r["weights"] - W).max() <= 1e-7 * max(1.0, np.abs(W).max()), s.req
        if r["kept"]:
            kept[s.req.key] = S
        nv = s.vol.shape[0]
        if nv:
            idx = np.sort(rng.choice(nv, size=min(n_points, nv), replace=False))
            pts = s.vol[torch.from_numpy(idx).to(s.vol.device)].double().cpu().numpy()
            ref = oracle.interpolate(s.xyz[S], W, s.radius, pts)
            got = s.out[torch.from_numpy(idx).to(s.out.device)].double().cpu().numpy()
            assert np.abs(got - ref).max() <= TOL_ORACLE * md, (s.req, np.abs(got - ref).max() / md)
    return stats


def test_served_requests_match_the_oracle():
    """Continuous batching with resident meshes: each served selection and its Eq. 6 output
    agree with the oracle run on that request alone (warm starts included)."""
    items = small_stream(14, 0.4)
    pool = serving.volume_pool(40_000, "cuda")
    with gcb.Server(0, hbm_budget=4 << 30, max_active=8) as srv:
        served = serving.replay(srv, items, pool, nv_per_nb=6, iterations=8, record=True)
    stats = check_against_oracle(served)
    assert stats["warm"] > 0 and stats["same"] + stats["certified"] == len(served), stats


def test_one_at_a_time_matches_the_oracle():
    items = small_stream(5, 0.0)
    pool = serving.volume_pool(40_000, "cuda")
    with gcb.Server(0, hbm_budget=4 << 30, max_active=1, flags=0) as srv:
        served = serving.replay(srv, items, pool, nv_per_nb=6, record=True)
    check_against_oracle(served)


def test_one_at_a_time_equals_alone():
    items = small_stream(6, 0.0)
    pool = serving.volume_pool(40_000, "cuda")
    with gcb.Server(0, hbm_budget=4 << 30, max_active=1, flags=0) as srv:
        served = serving.replay(srv, items, pool, nv_per_nb=6)
        assert not any(s.result["warm"] or s.result["kept"] for s in served)
        # one at a time: each admission waits for the previous output
        adm = sorted((s.result["t_admit"], s.result["t_done"]) for s in served)
        assert all(adm[i + 1][0] >= adm[i][1] - 1e-4 for i in range(len(adm) - 1))
        check_same(served)


def test_small_budget_queues_and_evicts():
    items = small_stream(16, 0.5, scale=0.15)
    pool = serving.volume_pool(40_000, "cuda")
    budget = 48 << 20
    with gcb.Server(0, hbm_budget=budget, max_active=8) as srv:
        served = serving.replay(srv, items, pool, nv_per_nb=4, iterations=8)
        used, resident = srv.memory()
        assert resident <= len({s.req.key for s in served})
        # idle resident meshes were evicted to stay within the budget
        assert used <= budget or resident == 1, (used, resident)
        check_same(served)


def test_bad_request_rejected():
    with gcb.Server(0, hbm_budget=1 << 30, max_active=2) as srv:
        with pytest.raises(gcb.GcbError) as e:
            srv.submit(np.zeros((2, 3)), np.zeros((2, 3)), 1.0, 1, 0.0)
        assert e.value.code == gcb.GCB_E_INVALID
        assert srv.progress(4) == 0


def test_mixed_dtypes_in_one_round():
    """Requests with FP32 and FP64 volume arrays finishing together: one batched volume launch
    per dtype pair; each output equals its own deformation alone."""
    items = small_stream(8, 0.0)
    pool64 = serving.volume_pool(20_000, "cuda")
    with gcb.Server(0, hbm_budget=4 << 30, max_active=8) as srv:
        served = []
        for n, (req, base, disp, tol) in enumerate(items):
            dt = torch.float32 if n % 2 else torch.float64
            vol = pool64[req.key % 2][: 4 * base.nb].to(dt).contiguous()
            out = torch.empty_like(vol)
            tk = srv.submit(base.xyz, disp, base.radius, base.m, tol, seed=base.seed, mesh_key=-1, vol=vol, out=out)
            served.append((tk, base, disp, tol, vol, out))
        while srv.progress(16):
            pass
        torch.cuda.synchronize()
        for tk, base, disp, tol, vol, out in served:
            r = srv.result(tk)
            assert r["state"] == 3 and not r["warm"] and not r["kept"]
            c = gcb.Context(0)
            c.set_boundary(base.xyz, disp)
            c.set_params(base.radius, base.m, tol, seed=base.seed)
            c.select()
            ref = c.deform(vol, out_dtype=vol.dtype)
            torch.cuda.synchronize()
            md = float(np.sqrt((disp ** 2).sum(axis=1)).max())
            assert (out.double() - ref.double()).abs().max().item() <= TOL_SAME * md
            c.close()


def test_forget_finished_tickets_only():
    """A queued ticket cannot be forgotten; a finished one can, and is unknown afterwards."""
    items = small_stream(3, 0.0)
    pool64 = serving.volume_pool(20_000, "cuda")
    with gcb.Server(0, hbm_budget=4 << 30, max_active=1) as srv:
        tickets = []
        for req, base, disp, tol in items:
            vol = pool64[req.key % 2][: 4 * base.nb].contiguous()
            out = torch.empty_like(vol)
            tickets.append((srv.submit(base.xyz, disp, base.radius, base.m, tol, seed=base.seed, vol=vol, out=out),
                            vol, out))
        with pytest.raises(gcb.GcbError) as e:
            srv.forget(tickets[-1][0])            # still queued
        assert e.value.code == gcb.GCB_E_STATE
        while srv.progress(16):
            pass
        torch.cuda.synchronize()
        for tk, _, _ in tickets:
            assert srv.result(tk)["state"] == 3
            srv.forget(tk)
            with pytest.raises(gcb.GcbError) as e:
                srv.result(tk)
            assert e.value.code == gcb.GCB_E_INVALID
