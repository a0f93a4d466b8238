"""Batched persistent launches and the continuous-batching server on the GPU.

Every lattice advanced in a batch or by the server must give exactly the
result of the same lattice advanced alone by the single-lattice kernel with
the same vector width: the per-site arithmetic is identical and there are no
atomics, so the comparison is bitwise.  The batch results are also checked
against the FP64 oracle with the FP32 bar of the parity tests.
"""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1007_3109_amd import workloads  # noqa: E402

if torch.cuda.is_available():
    from paper_1007_3109_amd import lbrd  # noqa: E402



def log(msg):
    print(msg, flush=True)


def solo(cfg, rho0, steps):
    """A single solver with its default launch shape (several steps per
    launch): the batched and served results must equal it bitwise."""
    s = lbrd.Solver(cfg)
    s.set_tuning(graph_steps=0)
    s.init(rho0).step(steps)
    return s.moments()[0]


def mixed_cases():
    rng = np.random.default_rng(0)
    cases = []
    for j, (side, storage) in enumerate([(48, "f32"), (67, "f32"), (128, "f16"), (33, "bf16"), (200, "f32"),
                                         (20, "f64"), (96, "f16")]):
        if j % 3 == 2:
            cfg = lbrd.make_config(side, side + 3, 1, tau=0.8, storage=storage, reaction="linear", K=[[-0.003]],
                                   rho_ref=(1.0,))
            rho0 = workloads.sinusoid(side, side + 3, 0.1, 1)
        else:
            F, k = workloads.draw_gs_unstable(rng)
            cfg = lbrd.make_config(side, side + 3, 2, tau=workloads.GS_TAU, storage=storage, reaction="gray_scott",
                                   F=F, k=k, rho_ref=(1.0, 0.0))
            rho0 = workloads.gray_scott_square(side, side + 3, rng=np.random.default_rng(j))
        cases.append((cfg, rho0))
    return cases


@pytest.mark.parametrize("mode", ["default", "one-step", "three-step"])
def test_batch_gs_f32_equals_solo_and_oracle(mode):
    """The batched Gray-Scott FP32 job (default: five steps per launch on
    32 x 10 LDS tiles inside the Infinity Cache, graphs of 30 steps; also
    persistent one-step launches and three steps per launch) equals solo runs
    bitwise after 151 steps (graph replays plus a ragged remainder) and the
    FP64 oracle within the FP32 floor."""
    insts = [i for i in workloads.batch_sweep(3, grid=4, sides=(64, 96, 130))]
    cfgs = [lbrd.make_config(i.side, i.side, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott",
                             F=i.F, k=i.k) for i in insts]
    b = lbrd.Batch(cfgs)
    t = b.tuning()
    assert (t.fused_steps, t.tile_cols, t.tile_rows, t.graph_steps) == (5, 32, 10, 30)
    if mode == "one-step":
        b.set_tuning(fused_steps=1, waves=4, blocks_per_cu=8, graph_steps=16)
    elif mode == "three-step":
        b.set_tuning(fused_steps=3, tile_rows=4, tile_cols=64, waves=8, graph_steps=18)
        with pytest.raises(lbrd.LbrdError):
            b.set_tuning(graph_steps=16)        # not an even number of three-step launches
    for idx, inst in enumerate(insts):
        b.init(idx, workloads.batch_initial(inst))
    steps = 151
    b.step(steps)
    for idx, inst in enumerate(insts):
        got = b.moments(idx)[0]
        want = solo(cfgs[idx], workloads.batch_initial(inst), steps)
        assert torch.equal(got, want), idx
        if idx % 5 == 0:
            r0 = workloads.batch_initial(inst)
            kw = dict(F=inst.F, k=inst.k)
            ref = oracle.solve(r0, steps, list(workloads.GS_TAU), oracle.REACT_GRAY_SCOTT, **kw)
            floor = oracle.rel_l2(oracle.solve(r0, steps, list(workloads.GS_TAU), oracle.REACT_GRAY_SCOTT,
                                               precision="f32", **kw), ref)
            tol = np.where(floor <= 1e-6, 1e-5, 3 * floor)
            assert np.all(oracle.rel_l2(got.cpu().numpy(), ref) <= tol)
    log(f"batch of {len(insts)} GS f32 lattices ({mode}): bitwise equal to solo runs")


def test_full_size_sweep_batch_sampled():
    """The benchmark's batched workload at full size (256 Gray-Scott instances,
    sides 128..512, seed 0, 4.2 GB of buffers, default launch shape: nine
    steps per launch on marching strips of 128 rows, graphs of 36 steps):
    after 70 steps (one graph replay and a ragged remainder) a sample of
    instances equals their solo runs bitwise, and the smallest sampled
    lattice equals the FP64 oracle within the FP32 floor."""
    insts = workloads.batch_sweep(0)
    cfgs = [lbrd.make_config(i.side, i.side, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott",
                             F=i.F, k=i.k) for i in insts]
    b = lbrd.Batch(cfgs)
    t = b.tuning()
    assert (t.fused_steps, t.march_rows, t.waves, t.graph_steps) == (9, 128, 4, 36)
    for idx, inst in enumerate(insts):
        b.init(idx, workloads.batch_initial(inst))
    steps = 70
    b.step(steps)
    sample = [0, 37, 101, 128, 200, 255]
    for idx in sample:
        got = b.moments(idx)[0]
        assert torch.equal(got, solo(cfgs[idx], workloads.batch_initial(insts[idx]), steps)), idx
    small = min(sample, key=lambda i: insts[i].side)
    r0 = workloads.batch_initial(insts[small])
    kw = dict(F=insts[small].F, k=insts[small].k)
    ref = oracle.solve(r0, steps, list(workloads.GS_TAU), oracle.REACT_GRAY_SCOTT, **kw)
    floor = oracle.rel_l2(oracle.solve(r0, steps, list(workloads.GS_TAU), oracle.REACT_GRAY_SCOTT, precision="f32",
                                       **kw), ref)
    tol = np.where(floor <= 1e-6, 1e-5, 3 * floor)
    assert np.all(oracle.rel_l2(b.moments(small)[0].cpu().numpy(), ref) <= tol)
    log(f"full-size sweep batch: {len(insts)} instances, sampled {sample} bitwise equal to solo runs")
    b.close()


def serve_mix_cases():
    """F32 / F16 / BF16 storage, single-species decay or Gray-Scott: the
    serving mix, which batches with several steps per launch."""
    return [(c, r) for c, r in mixed_cases() if c.storage != lbrd.STORAGE["f64"]]


@pytest.mark.parametrize("ts,cols,graph_steps,nt", [(4, 64, 0, 0), (4, 64, 16, 1), (3, 64, 12, 0), (2, 32, 4, 1),
                                                   (5, 32, 10, 0), (7, 32, 28, 1), (8, 64, 0, 0)])
def test_batch_multi_step_advance_equals_solo(ts, cols, graph_steps, nt):
    """Per-instance step counts (lbrd_batch_advance) on the serving mix with
    T steps per launch: counts that are not multiples of T end with a shorter
    launch (down to a single step), instances with 0 steps stay put, and every
    instance equals its solo run bitwise."""
    cases = serve_mix_cases()
    b = lbrd.Batch([c for c, _ in cases])
    b.set_tuning(fused_steps=ts, tile_rows=4, tile_cols=cols, waves=8, blocks_per_cu=0, graph_steps=graph_steps,
                 nontemporal=nt)
    for idx, (_, rho0) in enumerate(cases):
        b.init(idx, rho0)
    counts = [1, 2, 3, 0, 5, 23][:len(cases)]
    b.advance(counts)
    more = [7, 0, 1, 4, 30, 2][:len(cases)]
    b.advance(more)
    b.step(9)
    for idx, (cfg, rho0) in enumerate(cases):
        n = counts[idx] + more[idx] + 9
        assert b.time(idx) == n
        assert torch.equal(b.moments(idx)[0], solo(cfg, rho0, n)), (idx, n)
    with pytest.raises(lbrd.LbrdError):                 # at most eight steps per launch, 32 or 64 columns
        b.set_tuning(fused_steps=9, tile_rows=4, waves=8, blocks_per_cu=0, graph_steps=0)
    with pytest.raises(lbrd.LbrdError):
        b.set_tuning(fused_steps=4, tile_rows=4, tile_cols=128, waves=8, blocks_per_cu=0, graph_steps=0)


def march_cases():
    """The serving mix plus lattices smaller than a strip or a segment (1 x 1,
    2 x 3, 45 x 70), where strips wrap around the lattice."""
    extra = []
    for j, (nx, ny, storage) in enumerate([(1, 1, "f32"), (2, 3, "f16"), (45, 70, "bf16")]):
        F, k = workloads.draw_gs_unstable(np.random.default_rng(40 + j))
        cfg = lbrd.make_config(nx, ny, 2, tau=workloads.GS_TAU, storage=storage, reaction="gray_scott", F=F, k=k,
                               rho_ref=(1.0, 0.0))
        extra.append((cfg, workloads.gray_scott_square(nx, ny, rng=np.random.default_rng(50 + j))))
    return serve_mix_cases() + extra


@pytest.mark.parametrize("ts,rows,waves,bpc,graph_steps", [(2, 1, 1, 0, 0), (3, 7, 2, 1, 6), (5, 64, 4, 0, 10),
                                                           (7, 64, 4, 2, 28), (8, 16, 4, 0, 0), (6, 33, 1, 3, 12),
                                                           (4, 200, 4, 1, 8), (10, 128, 4, 0, 20),
                                                           (12, 9, 1, 1, 24), (11, 300, 4, 0, 0)])
def test_batch_march_advance_equals_solo(ts, rows, waves, bpc, graph_steps):
    """Batched marching strips (march_rows > 0) on the serving mix, T steps per
    launch, one wave per strip segment or a persistent grid: per-instance
    step counts that are not multiples of T end with a launch of fewer steps
    (the wider strip's halo covers them), instances with 0 steps stay put,
    and every instance equals its solo run bitwise."""
    cases = march_cases()
    b = lbrd.Batch([c for c, _ in cases])
    b.set_tuning(fused_steps=ts, march_rows=rows, waves=waves, blocks_per_cu=bpc, graph_steps=graph_steps,
                 nontemporal=int(ts % 2 == 0))
    t = b.tuning()
    assert (t.fused_steps, t.march_rows, t.tile_cols, t.tile_rows) == (ts, rows, 0, 0)
    for idx, (_, rho0) in enumerate(cases):
        b.init(idx, rho0)
    counts = [1, 2, 3, 0, 5, 23, 7, 11, 4][:len(cases)]
    b.advance(counts)
    more = [7, 0, 1, 4, 30, 2, 9, 1, 13][:len(cases)]
    b.advance(more)
    b.step(9)
    for idx, (cfg, rho0) in enumerate(cases):
        n = counts[idx] + more[idx] + 9
        assert b.time(idx) == n
        assert torch.equal(b.moments(idx)[0], solo(cfg, rho0, n)), (idx, n)
    with pytest.raises(lbrd.LbrdError):                 # one, two or four waves per workgroup
        b.set_tuning(fused_steps=4, march_rows=8, waves=8, blocks_per_cu=0, graph_steps=0)
    with pytest.raises(lbrd.LbrdError):                 # at most 12 steps per launch on marching strips
        b.set_tuning(fused_steps=13, march_rows=8, waves=4, blocks_per_cu=0, graph_steps=0)
    log(f"batched marching T {ts}, {rows} rows, {waves} waves, blocks per CU {bpc}: {len(cases)} instances bitwise "
        f"equal to solo runs")
    b.close()


def test_batch_march_gray_scott_set_equals_solo():
    """The FP32 Gray-Scott batch set on marching strips (the default beyond
    the Infinity Cache), nine instances of sides 64 and 96 with a graph of 14
    steps and a ragged remainder: every instance equals its solo run
    bitwise."""
    insts = workloads.batch_sweep(2, grid=3, sides=(64, 96))
    cfgs = [lbrd.make_config(i.side, i.side, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott",
                             F=i.F, k=i.k) for i in insts]
    b = lbrd.Batch(cfgs)
    b.set_tuning(fused_steps=7, march_rows=64, waves=4, blocks_per_cu=0, graph_steps=14)
    for idx, inst in enumerate(insts):
        b.init(idx, workloads.batch_initial(inst))
    b.step(33)
    for idx, inst in enumerate(insts):
        assert torch.equal(b.moments(idx)[0], solo(cfgs[idx], workloads.batch_initial(inst), 33)), idx
    b.close()


@pytest.mark.parametrize("graph_steps", [0, 8])
def test_batch_mixed_storage_and_reactions(graph_steps):
    cases = mixed_cases()
    b = lbrd.Batch([c for c, _ in cases])
    b.set_tuning(graph_steps=graph_steps)
    for idx, (_, rho0) in enumerate(cases):
        b.init(idx, rho0)
    b.step(37)
    b.step(20)
    for idx, (cfg, rho0) in enumerate(cases):
        got = b.moments(idx)[0]
        assert torch.equal(got, solo(cfg, rho0, 57)), idx


def test_batch_with_advected_instances_equals_solo():
    """Instances with an equilibrium velocity batch through the persistent
    one-step kernel (any variant): advected Gray-Scott in FP32, an advected
    single species in F16, and a plain Gray-Scott lattice; each equals its
    solo run bitwise, also with per-instance step counts."""
    rng = np.random.default_rng(9)
    F, k = workloads.draw_gs_unstable(rng)
    cases = [
        (lbrd.make_config(70, 50, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott", F=F, k=k,
                          u=(0.1, -0.04)), workloads.gray_scott_square(70, 50, rng=np.random.default_rng(1))),
        (lbrd.make_config(64, 33, 1, tau=0.8, storage="f16", reaction="linear", K=[[-0.002]], rho_ref=(1.0,),
                          u=(-0.05, 0.12)), workloads.sinusoid(64, 33, 0.1, 2)),
        (lbrd.make_config(96, 96, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott", F=F, k=k),
         workloads.gray_scott_square(96, 96, rng=np.random.default_rng(2))),
    ]
    b = lbrd.Batch([c for c, _ in cases])
    assert b.tuning().fused_steps == 1
    for idx, (_, rho0) in enumerate(cases):
        b.init(idx, rho0)
    counts = [41, 17, 30]
    b.advance(counts)
    for idx, (cfg, rho0) in enumerate(cases):
        assert torch.equal(b.moments(idx)[0], solo(cfg, rho0, counts[idx])), idx


def test_batch_autotune_then_run():
    insts = workloads.batch_sweep(1, grid=3, sides=(64, 128))
    cfgs = [lbrd.make_config(i.side, i.side, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott",
                             F=i.F, k=i.k) for i in insts]
    b = lbrd.Batch(cfgs)
    t = b.autotune(steps=3)
    if t.fused_steps == 1:
        assert 1 <= t.blocks_per_cu <= 32 and t.waves in (1, 2, 4)
    elif t.march_rows > 0:
        assert 4 <= t.fused_steps <= 12 and t.march_rows in (16, 32, 64, 128, 256) and t.waves in (1, 4)
        assert t.graph_steps % (2 * t.fused_steps) == 0
    else:
        assert 2 <= t.fused_steps <= 8 and t.tile_cols in (32, 64) and t.tile_rows in (4, 8, 12, 16, 20)
        assert t.graph_steps % (2 * t.fused_steps) == 0
    log(f"batch autotune chose {t.as_dict()}")
    assert lbrd.lib.lbrd_batch_step(b._h, 1) == lbrd.ESTATE
    for idx, inst in enumerate(insts):
        b.init(idx, workloads.batch_initial(inst))
    b.step(40)
    for idx, inst in enumerate(insts):
        assert torch.equal(b.moments(idx)[0], solo(cfgs[idx], workloads.batch_initial(inst), 40))


def test_server_results_equal_solo_runs():
    """The serving mix (seven steps per launch inside the server's rounds):
    request lengths that are not multiples of the chunk or of seven, including
    a single step, equal their solo runs bitwise."""
    cases = serve_mix_cases()
    steps = [130, 64, 300, 1, 77, 250]
    srv = lbrd.Server(arena_bytes=256 << 20, chunk_steps=64)
    tickets = []
    for (cfg, rho0), n in zip(cases, steps):
        tickets.append(srv.submit(cfg, rho0, n))
    for t in tickets:
        srv.wait(t, 120)
    for t, (cfg, rho0), n in zip(tickets, cases, steps):
        rho, mass, info = srv.take(t)
        want = solo(cfg, rho0, n).cpu().numpy()
        assert np.array_equal(rho, want), t
        assert info.state == 2 and info.done_s >= info.admit_s >= info.submit_s
        np.testing.assert_allclose(mass, want.reshape(want.shape[0], -1).sum(axis=1), rtol=1e-12)
    st = srv.stats()
    assert st.completed == len(tickets) and st.resident == 0 and st.queued == 0
    srv.close()


def test_server_rounds_beyond_the_cache_equal_solo_runs():
    """Rounds whose resident buffers exceed the Infinity Cache run on
    marching strips, the others on LDS tiles: two 2048^2 FP32 Gray-Scott
    requests (1.2 GB of buffers together) beside small ones of the serving
    mix; once the large ones finish the rounds go back to LDS tiles.  Every
    result equals its solo run bitwise."""
    big = []
    for j in range(2):
        F, k = workloads.draw_gs_unstable(np.random.default_rng(70 + j))
        cfg = lbrd.make_config(2048, 2048, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott", F=F, k=k)
        big.append((cfg, workloads.gray_scott_square(2048, 2048, rng=np.random.default_rng(80 + j))))
    cases = big + serve_mix_cases()
    steps = [23, 9] + [130, 64, 300, 1, 77, 250][:len(cases) - 2]
    srv = lbrd.Server(arena_bytes=3 << 30, chunk_steps=64)
    tickets = [srv.submit(cfg, rho0, n) for (cfg, rho0), n in zip(cases, steps)]
    for t in tickets:
        srv.wait(t, 300)
    for t, (cfg, rho0), n in zip(tickets, cases, steps):
        rho, _, info = srv.take(t)
        assert info.state == 2
        assert np.array_equal(rho, solo(cfg, rho0, n).cpu().numpy()), (t, cfg.nx, n)
    srv.close()
    log(f"server: {len(cases)} requests, two of them 2048^2 (marching rounds), bitwise equal to solo runs")


def test_server_with_an_advected_request_equals_solo():
    """A request with an equilibrium velocity sends its rounds through the
    one-step kernel of the any-variant set; results still equal solo runs."""
    cfg_a = lbrd.make_config(80, 60, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott",
                             F=workloads.GS_F, k=workloads.GS_K, u=(0.07, 0.03))
    cfg_b = lbrd.make_config(48, 48, 1, tau=0.9, storage="f32", reaction="linear", K=[[-0.001]])
    r_a = workloads.gray_scott_square(80, 60, seed=5)
    r_b = workloads.sinusoid(48, 48, 0.1, 1)
    srv = lbrd.Server(arena_bytes=64 << 20, chunk_steps=40)
    ta = srv.submit(cfg_a, r_a, 97)
    tb = srv.submit(cfg_b, r_b, 55)
    for t in (ta, tb):
        srv.wait(t, 120)
    for t, cfg, r0, n in ((ta, cfg_a, r_a, 97), (tb, cfg_b, r_b, 55)):
        rho, _, info = srv.take(t)
        assert info.state == 2
        assert np.array_equal(rho, solo(cfg, r0, n).cpu().numpy()), t
    srv.close()


def test_server_destroy_with_queued_requests():
    """Destroying a server finishes the resident request and drops the queued
    ones: the call returns promptly and the resident work stays consistent."""
    import time

    cfg = lbrd.make_config(128, 128, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott", F=0.04, k=0.06)
    fp = lbrd.server_footprint(cfg)
    srv = lbrd.Server(arena_bytes=int(1.5 * fp) + (4 << 20), chunk_steps=100)
    rho0 = workloads.gray_scott_square(128, 128, seed=1)
    tickets = [srv.submit(cfg, rho0, 2000) for _ in range(5)]
    assert len(set(tickets)) == 5
    t0 = time.perf_counter()
    srv.close()
    assert time.perf_counter() - t0 < 30


def test_server_admission_by_footprint():
    """An arena that holds about two requests at a time: the others queue and
    are admitted as memory frees; all finish; the peak stays within the arena."""
    cfg = lbrd.make_config(256, 256, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott", F=0.04, k=0.06)
    fp = lbrd.server_footprint(cfg)
    arena = int(2.5 * fp) + (1 << 20)
    srv = lbrd.Server(arena_bytes=arena, chunk_steps=50)
    rho0 = workloads.gray_scott_square(256, 256, seed=0)
    tickets = [srv.submit(cfg, rho0, 120) for _ in range(6)]
    for t in tickets:
        srv.wait(t, 120)
    outs = [srv.take(t) for t in tickets]
    for rho, _, info in outs[1:]:
        assert np.array_equal(rho, outs[0][0])
    admits = sorted(o[2].admit_s for o in outs)
    assert admits[-1] > admits[1]            # later requests waited for memory
    st = srv.stats()
    assert st.arena_peak_used <= st.arena_bytes and st.arena_peak_used >= 2 * fp
    big = lbrd.make_config(2048, 2048, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott", F=0.04, k=0.06)
    with pytest.raises(lbrd.LbrdError) as ei:
        srv.submit(big, np.zeros((2, 2048, 2048)), 10)
    assert ei.value.status == lbrd.ENOMEM
    srv.close()
