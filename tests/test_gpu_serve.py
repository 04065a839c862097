"""GPU tests of the continuous-batching server: every request's answer is
the same alone and in the mix; captured-graph replays at changing live counts
match eager runs; the server's outputs match the FP64 oracle; a tight HBM
budget still serves everything; timeouts and cancellation leave the queue."""

import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_common import BF16_TOL_MAG, FP32_TOL_MAG, filters6, ssp_large

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_06830_amd.serve as S
    return S


@pytest.fixture(scope="module")
def handles(S):
    import paper_2112_06830_amd as P
    return (P.SspBlock.from_synth(ssp_large(), precisions=("fp32", "bf16")),
            P.FilterBank.from_synth(filters6()), synth.population.make_time_grid(100))


@pytest.fixture(scope="module")
def engine(S, handles):
    _say("serve engine: capturing slots")
    eng = S.ServeEngine(*handles, buckets=(2048, 8192, 32768), hbm_budget_bytes=8 << 30,
                        batch_galaxies={S.KIND_GRAD: 8192})
    eng.start()
    yield eng
    eng.stop()


def _alone(eng, r):
    """The same request through the plain calls, on its own."""
    import torch
    import paper_2112_06830_amd as P
    d = torch.device("cuda")
    pop = P.DevicePopulation(eng.t_table, None, torch.tensor(r.sfh_params, device=d),
                             *(torch.tensor(getattr(r, k), device=d) for k in
                               ("z", "lgmet", "sigma_z", "av", "delta", "bump")))
    if r.grad:
        m, g = P.mags_residual_vjp(eng.ssp, eng.flt, eng.cosmo, pop,
                                   torch.tensor(r.targets, device=d),
                                   want=("sfh_params", "lgmet", "sigma_z", "av", "delta", "bump"))
        return m.cpu().numpy(), {k: v.cpu().numpy() for k, v in g.items()}
    m = P.mags(eng.ssp, eng.flt, eng.cosmo, pop, precision="bf16")
    return m.cpu().numpy(), None


def test_alone_equals_in_the_mix(S, engine):
    t, reqs = S.make_trace(24, rate_hz=400.0, seed=11, n_range=(300, 20000))
    _say(f"serve 24 requests, {sum(r.n for r in reqs)} galaxies")
    S.replay_trace(engine, t, reqs, timeout_s=120)
    assert sum(engine.stats["batches"].values()) >= 2
    assert engine.stats["captures_in_loop"] == 0 and engine.stats["evictions"] == 0
    for r in reqs:
        assert r.error is None
        m_alone, g_alone = _alone(engine, r)
        assert np.array_equal(r.mags, m_alone), r.rid
        if r.grad:
            for k, v in g_alone.items():
                assert np.array_equal(r.grads[k], v), (r.rid, k)


def test_served_results_match_oracle(S, engine):
    t, reqs = S.make_trace(6, rate_hz=100.0, seed=12, n_range=(200, 3000), grad_fraction=0.5)
    _say("serve 6 requests vs oracle")
    S.replay_trace(engine, t, reqs, timeout_s=120)
    ssp, flt = ssp_large(), filters6()
    for r in reqs:
        idx = np.arange(0, r.n, max(1, r.n // 6))[:6]
        pop = synth.Population(
            t_table=synth.population.make_time_grid(100), sfh_params=r.sfh_params[:, idx],
            z=r.z[idx].astype(np.float64), lgmet=r.lgmet[idx].astype(np.float64),
            sigma_z=r.sigma_z[idx].astype(np.float64), av=r.av[idx].astype(np.float64),
            delta=r.delta[idx].astype(np.float64), bump=r.bump[idx].astype(np.float64),
            targets=np.zeros((idx.size, 6)))
        inp = oracle.prepare_inputs(ssp, flt, pop)
        ref = oracle.mags(inp)
        tol = FP32_TOL_MAG if r.grad else BF16_TOL_MAG
        assert np.max(np.abs(r.mags[idx] - ref)) < tol, r.rid
        if r.grad:
            bar = 2.0 * (r.mags[idx].astype(np.float64) - r.targets[idx])
            g = oracle.mags_vjp(inp, bar)
            for k, rk in (("lgmet", "lgmet_bar"), ("av", "av_bar"), ("delta", "delta_bar")):
                ref_g = g[rk]
                err = np.abs(r.grads[k][idx] - ref_g)
                assert np.all(err <= 1e-3 * np.maximum(np.abs(ref_g), 1e-2 * np.sqrt(np.mean(ref_g**2)))), (r.rid, k)


def test_graph_replays_match_eager(S, engine):
    """Replay one captured gradient slot on batches of different live counts,
    with eager work and synchronisation between replays; each replay must
    equal the eager launch sequence on the same inputs, and rows past the
    live count must keep what they held."""
    import torch
    _say("graph replay vs eager at changing live counts")
    slot = S._Slot(engine, S.KIND_GRAD, 2048)
    stream = torch.cuda.Stream()
    slot.capture(stream)
    assert slot.graph is not None
    for seed, n_range in ((1, (500, 900)), (2, (200, 300)), (3, (700, 1000))):
        _, reqs = S.make_trace(2, seed=100 + seed, n_range=n_range, grad_fraction=1.0)
        par, in32, tgt = slot.h_par.numpy(), slot.h_in32.numpy(), slot.h_tgt.numpy()
        o = 0
        for r in reqs:
            par[:, o:o + r.n] = r.sfh_params
            for i, k in enumerate(("z", "lgmet", "sigma_z", "av", "delta", "bump")):
                in32[i, o:o + r.n] = getattr(r, k)
            tgt[o:o + r.n] = r.targets
            o += r.n
        slot.h_live[0] = o
        slot.d_par.copy_(slot.h_par)
        slot.d_in32.copy_(slot.h_in32)
        slot.d_tgt.copy_(slot.h_tgt)
        slot.d_live.copy_(slot.h_live)
        slot.mags.fill_(-1.0)
        with torch.cuda.stream(stream):
            slot.graph.replay()
        stream.synchronize()
        rep = (slot.mags[:o].clone(), slot.g64[:, :o].clone(), slot.g32[:, :o].clone())
        assert bool((slot.mags[o:] == -1.0).all())          # padding rows untouched
        _ = torch.ones(1000, device="cuda").sum().item()   # unrelated eager work
        with torch.cuda.stream(stream):
            slot.run_body()
        stream.synchronize()
        assert torch.equal(rep[0], slot.mags[:o])
        assert torch.equal(rep[1], slot.g64[:, :o])
        assert torch.equal(rep[2], slot.g32[:, :o])


def test_tight_budget_still_serves(S, handles):
    _say("serve with a two-slot HBM budget")
    eng = S.ServeEngine(*handles, buckets=(2048, 8192), hbm_budget_bytes=1)
    # the smallest budget that holds one 8192-slot of each kind
    need = eng.planner.slot_bytes("grad", 8192) + eng.planner.slot_bytes("fwd", 8192)
    eng.planner.budget = need
    eng.start()
    try:
        assert eng.stats["captures_in_warm"] == 2
        t, reqs = S.make_trace(10, rate_hz=1000.0, seed=13, n_range=(1000, 6000))
        S.replay_trace(eng, t, reqs, timeout_s=120)
        assert all(r.error is None for r in reqs)
        assert eng.planner.reserved <= eng.planner.budget
    finally:
        eng.stop()


def test_timeout_and_cancel(S, handles):
    _say("serve: cancelled and timed-out requests leave the queue")
    eng = S.ServeEngine(*handles, buckets=(2048,), hbm_budget_bytes=8 << 30)
    eng.warm()
    _, reqs = S.make_trace(3, seed=14, n_range=(500, 1500), grad_fraction=0.0)
    ok, gone, late = reqs
    late.timeout_s = 0.0
    for r in reqs:
        eng.submit(r)
    assert eng.cancel(gone)                       # still queued: it will not run
    eng.start()
    try:
        for r in reqs:
            assert r.done.wait(60)
        assert ok.error is None and ok.mags is not None
        assert gone.error == "cancelled" and gone.mags is None
        assert "timed out" in late.error and late.mags is None
        assert not eng.cancel(ok)                 # finished: nothing to cancel
        assert eng.stats["dropped"] == 2
    finally:
        eng.stop()
