"""Marching wave strips (tuning march_rows > 0): T steps per launch with the
intermediate rows carried in registers.  Every site runs the one-step
kernel's arithmetic on the same stored inputs, so after any number of steps
every population is bitwise equal to one-step launches: checked for every
storage form and reaction variant, 2 .. 12 steps per launch (FP64 2 .. 8), several segment
lengths (1 row, a ragged one, more than the lattice), workgroup sizes, both
tile orders and streaming stores, on tiny lattices (where a strip wraps
around the lattice several times), ragged ones and wider ones."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1007_3109_amd import workloads  # noqa: E402

if torch.cuda.is_available():
    from paper_1007_3109_amd import lbrd  # noqa: E402

CASES = [("f64", "gray_scott", 2), ("f32", "gray_scott", 2), ("f16", "gray_scott", 2), ("bf16", "gray_scott", 2),
         ("f32", "linear", 1), ("f32", "linear", 3), ("f64", "linear", 4), ("f16", "linear", 1),
         ("f32", "gray_scott_advected", 2), ("bf16", "linear_advected", 1),
         ("f32", "gray_scott_shear", 2), ("f64", "linear_shear", 1)]


def _config(storage, reaction, ns, nx, ny):
    kw = dict(F=0.04, k=0.06) if reaction.startswith("gray_scott") else dict(K=-0.01 * np.eye(ns))
    if reaction.endswith("_advected"):
        kw["u"] = (0.09, -0.13)
    if reaction.endswith("_shear"):
        kw["u"] = (0.02, -0.04)
        kw["shear"] = (0.11, 2)
    return lbrd.make_config(nx, ny, ns, tau=[0.7, 1.2, 0.9, 0.8][:ns], storage=storage,
                            reaction=reaction.replace("_advected", "").replace("_shear", ""), rho_ref=(0.3,) * ns,
                            **kw)


@pytest.mark.parametrize("storage,reaction,ns", CASES)
def test_march_launch_is_bitwise_identical(storage, reaction, ns):
    ran = 0
    for ny, nx in [(1, 1), (3, 3), (2, 5), (45, 67), (33, 130), (17, 257), (70, 300)]:
        rng = np.random.default_rng(nx * 11 + ny)
        cfg = _config(storage, reaction, ns, nx, ny)
        f0 = rng.uniform(0.0, 0.1, size=(ns, 9, ny, nx))
        ref = lbrd.Solver(cfg)
        ref.set_tuning(fused_steps=1, graph_steps=0)
        ref.set_populations(f0).step(19)
        want = ref.get_populations()
        ref.close()
        s = lbrd.Solver(cfg)
        for steps in range(2, 9 if storage == "f64" else 13):
            for rows in (1, 7, 64):
                waves = (1, 2, 4)[ran % 3]
                s.set_tuning(fused_steps=steps, march_rows=rows, waves=waves, graph_steps=0,
                             nontemporal=int(ran % 5 == 0), plain_order=(ran // 3) % 2)
                s.set_populations(f0).step(19)
                assert torch.equal(s.get_populations(), want), (ny, nx, steps, rows, waves)
                ran += 1
        assert s.time() == 19
        s.close()
    print(f"march {storage} {reaction} N={ns}: {ran} shapes bitwise equal", flush=True)


def test_march_tuning_limits():
    cfg = _config("f32", "gray_scott", 2, 40, 30)
    s = lbrd.Solver(cfg)
    for bad in (dict(fused_steps=4, march_rows=-1), dict(fused_steps=4, march_rows=65537),
                dict(fused_steps=1, march_rows=-1), dict(fused_steps=13, march_rows=8),
                dict(fused_steps=9, march_rows=0)):
        with pytest.raises(lbrd.LbrdError):
            s.set_tuning(graph_steps=0, **bad)
    s.set_tuning(fused_steps=4, march_rows=65536, graph_steps=0)
    s.set_tuning(fused_steps=12, march_rows=8, graph_steps=0)   # marching: up to 12 steps a launch
    s.set_tuning(fused_steps=1, graph_steps=0)       # one-step launches ignore march_rows
    assert s.tuning().march_rows == 8 and s.tuning().fused_steps == 1
    s.close()
    d = lbrd.Solver(_config("f64", "gray_scott", 2, 40, 30))
    d.set_tuning(fused_steps=8, march_rows=8, graph_steps=0)
    with pytest.raises(lbrd.LbrdError):   # FP64 marching: at most 8
        d.set_tuning(fused_steps=9, march_rows=8, graph_steps=0)
    d.close()


@pytest.mark.parametrize("ts,rows,graph", [(4, 32, 8), (7, 64, 28), (8, 128, 16), (11, 342, 22)])
def test_march_with_graphs_and_oracle(ts, rows, graph):
    """Captured graphs of marching launches replayed between eager remainders
    equal plain one-step launches bitwise, and the FP64 oracle within 1e-5
    after 52 steps (Gray-Scott FP32 from the square start)."""
    rho0 = workloads.gray_scott_square(200, 160, seed=7)
    kw = dict(F=workloads.GS_F, k=workloads.GS_K)
    cfg = lbrd.make_config(200, 160, 2, tau=workloads.GS_TAU, storage="f32", reaction="gray_scott", **kw)
    a = lbrd.Solver(cfg)
    a.set_tuning(fused_steps=1, graph_steps=0)
    b = lbrd.Solver(cfg)
    b.set_tuning(fused_steps=ts, march_rows=rows, waves=4, graph_steps=graph)
    a.init(rho0)
    b.init(rho0)
    for n in (13, 6, 31, 2):
        a.step(n)
        b.step(n)
        assert torch.equal(a.moments()[0], b.moments()[0])
    ref = oracle.solve(rho0, 52, list(workloads.GS_TAU), oracle.REACT_GRAY_SCOTT, **kw)
    assert np.all(oracle.rel_l2(b.moments()[0].cpu().numpy(), ref) <= 1e-5)


@pytest.mark.parametrize("storage,reaction,ns,n,want_t,want_k", [
    ("f32", "gray_scott", 2, 4096, 10, 1), ("f32", "gray_scott", 2, 2048, 9, 1), ("f16", "gray_scott", 2, 4096, 8, 3),
    ("bf16", "gray_scott", 2, 2048, 6, 3), ("f32", "linear", 1, 4096, 11, 2), ("f64", "gray_scott", 2, 2048, 8, 1),
    ("f32", "gray_scott", 2, 1024, 7, 1)])
def test_default_segments_fill_k_waves_per_simd(storage, reaction, ns, n, want_t, want_k):
    """The default marching shape of a lattice beyond (or, FP32 from 1024^2,
    inside) the Infinity Cache: T steps per launch and segments of
    R = ceil(ny / floor(4 CUs k / strips)) rows, strips = ceil(nx / (64 -
    2(T-1))), so that strips x segments come to about k waves per SIMD."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    kw = dict(F=0.04, k=0.06) if reaction == "gray_scott" else dict(K=-0.01 * np.eye(ns))
    cfg = lbrd.make_config(n, n, ns, tau=[0.7, 1.2][:ns], storage=storage, reaction=reaction,
                           rho_ref=(1.0,) * ns, **kw)
    s = lbrd.Solver(cfg)
    t = s.tuning()
    s.close()
    strips = -(-n // (64 - 2 * (want_t - 1)))
    segs = max(1, 4 * cus * want_k // strips)
    assert (t.fused_steps, t.march_rows, t.waves) == (want_t, -(-n // segs), 4), t.as_dict()
    assert strips * -(-n // t.march_rows) <= 4 * cus * want_k
