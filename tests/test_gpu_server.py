"""GPU tests of the continuous-batching server (fge_server_* through the C ABI).

The server's contract: every request's F and B are exactly what fge_estimate_foreground gives for
that request alone (same kernels, same per-image plan; only the schedule differs), whatever else
shares its ticks; requests that arrive while others are on the device join the running ticks;
admitted footprints never exceed the budget.  The oracle check ties the served results to the
FP64 oracle at the storage type's tolerance.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2006_14970_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-4, "f16": 2e-3}

# Mixed sizes: whole-coarse-block images, tile-kernel levels only, and streaming finest levels.
SIZES = [(1500, 1000), (64, 48), (700, 1300), (257, 255), (33, 2000), (1024, 768), (130, 90),
         (1920, 1080), (400, 400), (2048, 300), (77, 1500), (999, 999), (1, 1), (640, 480),
         (1800, 1200), (96, 96), (3, 700), (1280, 720)]


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need an MI355X"
    from paper_2006_14970_amd import fge
    fge.load()
    return torch, fge


def make_inputs(torch, fge, params, sizes, seed0=6000):
    dt = fge.storage_dtype(params)
    out = []
    for k, (w, h) in enumerate(sizes):
        I, a = synth.smooth_device(w, h, seed0 + k, "cuda", dtype=dt)
        out.append((I, a))
    torch.cuda.synchronize()
    return out


def alone(torch, fge, params, inputs):
    res = []
    for I, a in inputs:
        F, B = fge.estimate_foreground(I, a, params)
        res.append((F, B))
    torch.cuda.synchronize()
    return res


def new_server(torch, fge, params, arena_gb=2.0, **cfg):
    arena = torch.empty(int(arena_gb * (1 << 30)), dtype=torch.uint8, device="cuda")
    return fge.Server(params, fge.server_config(**cfg), arena=arena)


def assert_same(torch, served, ref, what):
    for k, ((F, B), (Fr, Br)) in enumerate(zip(served, ref)):
        assert torch.equal(F, Fr) and torch.equal(B, Br), (what, k)


@pytest.mark.parametrize("storage", ["f16", "f32"])
def test_mixed_stream_matches_alone(gpu, storage):
    """Requests submitted while others run share ticks at different levels; each result equals
    the request run alone, bit for bit."""
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16 if storage == "f16" else fge.F32)
    inputs = make_inputs(torch, fge, p, SIZES)
    ref = alone(torch, fge, p, inputs)
    srv = new_server(torch, fge, p)
    served = []
    for k, (I, a) in enumerate(inputs):
        served.append(srv.submit(k, I, a))
        if k == 3:
            time.sleep(0.002)   # the first requests are on the device when the rest arrive
    srv.drain()
    done = srv.poll()
    st = srv.stats()
    srv.close()
    print(f"{storage}: {st}")
    assert sorted(r.id for r in done) == list(range(len(SIZES)))
    assert all(r.status == 0 for r in done)
    for r in done:
        assert r.admit_ms >= r.submit_ms - 1e-6 and r.latency_ms > 0 and r.ticks >= 1
    assert st["completed"] == st["submitted"] == len(SIZES)
    assert st["mixed_ticks"] > 0 and st["admitted_while_busy"] > 0
    assert_same(torch, served, ref, storage)


def test_served_results_match_oracle(gpu):
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16)
    sizes = [(300, 200), (64, 64), (257, 130), (1, 1), (90, 333)]
    inputs = make_inputs(torch, fge, p, sizes, seed0=6100)
    srv = new_server(torch, fge, p, arena_gb=0.25)
    served = [srv.submit(k, I, a) for k, (I, a) in enumerate(inputs)]
    srv.drain()
    srv.close()
    for (I, a), (F, B), (w, h) in zip(inputs, served, sizes):
        I64 = I.double().cpu().numpy()
        a64 = a.double().cpu().numpy()
        Fo, Bo = oracle.ml(I64, a64)
        err = max(float(np.abs(F.double().cpu().numpy() - Fo).max()),
                  float(np.abs(B.double().cpu().numpy() - Bo).max()))
        print(f"{w}x{h}: served f16 vs oracle {err:.2e}")
        assert err <= TOL["f16"], (w, h, err)


def test_serving_workload_sample_matches_oracle(gpu):
    """A 5% sample of the 2000-request serving workload: 100 requests drawn at random from the
    same stream (area log-uniform on 0.25-16 MP, aspect uniform on [0.5, 2], seed 5; inputs from
    the smooth generator with seed 5000 + request id, float16), served together under the default
    64 GB budget, each against the FP64 oracle on its float16 inputs."""
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16)
    reqs = synth.serving_requests(2000, seed=5)
    pick = sorted(np.random.Generator(np.random.PCG64(55)).choice(len(reqs), size=100,
                                                                  replace=False).tolist())
    inputs = []
    for i in pick:
        r = reqs[i]
        inputs.append(synth.smooth_device(r.W, r.H, 5000 + r.rid, "cuda", dtype=torch.float16))
    torch.cuda.synchronize()
    srv = new_server(torch, fge, p, arena_gb=8.0)
    served = [srv.submit(k, I, a) for k, (I, a) in enumerate(inputs)]
    srv.drain()
    done = srv.poll()
    srv.close()
    assert len(done) == len(pick) and all(d.status == 0 for d in done)
    worst, mp = 0.0, 0.0
    for (I, a), (F, B) in zip(inputs, served):
        Fo, Bo = oracle.ml(I.cpu().numpy().astype(np.float64), a.cpu().numpy().astype(np.float64),
                           parallel=True)
        err = max(float(np.abs(F.cpu().numpy().astype(np.float64) - Fo).max()),
                  float(np.abs(B.cpu().numpy().astype(np.float64) - Bo).max()))
        worst = max(worst, err)
        mp += a.numel() / 1e6
        assert err <= TOL["f16"], (tuple(a.shape), err)
    print(f"{len(pick)} sampled requests ({mp:.0f} MP): worst f16 max-abs vs oracle {worst:.2e}")


def test_budget_admission(gpu):
    """A budget that holds about two of the requests: admission waits for memory, the peak
    admitted footprint stays within the budget, and the results are unchanged."""
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16)
    sizes = SIZES[:10]
    inputs = make_inputs(torch, fge, p, sizes, seed0=6200)
    ref = alone(torch, fge, p, inputs)
    fp = sorted(fge.server_request_bytes(h, w, p) for w, h in sizes)
    budget = fp[-1] + fp[-2] + 4096
    srv = new_server(torch, fge, p, budget_bytes=budget)
    served = [srv.submit(k, I, a) for k, (I, a) in enumerate(inputs)]
    srv.drain()
    st = srv.stats()
    srv.close()
    print(st)
    assert st["peak_charged_bytes"] <= budget
    assert st["peak_active"] >= 2
    assert_same(torch, served, ref, "budget")


@pytest.mark.parametrize("cfg", [{"max_active": 1}, {"max_active": 3, "pipeline_depth": 1},
                                 {"tick_table_bytes": 64 << 10, "pipeline_depth": 4}])
def test_scheduler_limits(gpu, cfg):
    """One request at a time, shallow pipelines, and tick tables so small that requests are
    deferred to later ticks: the results stay those of the requests run alone."""
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16)
    sizes = SIZES[:12]
    inputs = make_inputs(torch, fge, p, sizes, seed0=6300)
    ref = alone(torch, fge, p, inputs)
    srv = new_server(torch, fge, p, **cfg)
    served = [srv.submit(k, I, a) for k, (I, a) in enumerate(inputs)]
    srv.drain()
    st = srv.stats()
    srv.close()
    if cfg.get("max_active") == 1:
        assert st["peak_active"] == 1
    assert_same(torch, served, ref, str(cfg))


def test_reuse_after_drain_and_rejections(gpu):
    torch, fge = gpu
    p = fge.default_params(storage=fge.F16)
    inputs = make_inputs(torch, fge, p, [(500, 400), (200, 100)], seed0=6400)
    ref = alone(torch, fge, p, inputs)
    budget = fge.server_request_bytes(400, 500, p)
    srv = new_server(torch, fge, p, arena_gb=0.25, budget_bytes=budget)
    for rnd in range(3):   # the arena and the slots are reused across drains
        served = [srv.submit(10 * rnd + k, I, a) for k, (I, a) in enumerate(inputs)]
        srv.drain()
        assert len(srv.poll()) == 2
        assert_same(torch, served, ref, f"round {rnd}")
    big = torch.zeros((3, 600, 600), dtype=torch.float16, device="cuda")
    with pytest.raises(fge.FgeError) as e:
        srv.submit(99, big, big[0])
    assert e.value.status == fge.FGE_EBUDGET
    with pytest.raises(fge.FgeError) as e:
        srv.submit_ptrs(98, 0, 0, 10, 10, 0, 0)
    assert e.value.status == fge.FGE_EINVAL
    srv.close()
    with pytest.raises(fge.FgeError) as e:
        new_server(torch, fge, fge.default_params(coarse_max_px=-1), arena_gb=0.01)
    assert e.value.status == fge.FGE_EUNSUPPORTED
