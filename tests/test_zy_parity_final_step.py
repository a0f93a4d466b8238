"""The 1024^2 Gray-Scott workload in FP32 storage against the FP64 oracle up to
its final step (20000), in the launch configuration the benchmark times.

Gray-Scott with F = 0.04, k = 0.06, tau = (1.0, 0.75) (D_u/D_v = 2), the
square start with seeded U(-0.01, 0.01) noise (Section IV start), the update of
Section II.A (second Eq. "relax").  At each checkpoint n the tolerance follows
the FP32 rule: relative L2 <= 1e-5 where the oracle's own float build stays
within 1e-6 of FP64 (its rounding floor F(n)), else <= 3 F(n): the pattern
dynamics amplify any rounding difference with time, so after thousands of
steps the floor of a plain float implementation sets the bar.

The oracle runs both builds over the whole lattice (about 4e10 species-site
updates each), several minutes on the host's cores.
"""
from __future__ import annotations

import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1007_3109_amd import workloads  # noqa: E402

if torch.cuda.is_available():
    from paper_1007_3109_amd import lbrd  # noqa: E402


@pytest.mark.timeout(1500)
def test_gray_scott_1024_checkpoints_to_final_step():
    n, seed = 1024, 0
    rho0 = workloads.gray_scott_square(n, n, seed=seed)
    kw = dict(F=workloads.GS_F, k=workloads.GS_K)
    taus = list(workloads.GS_TAU)
    s = lbrd.Solver(lbrd.make_config(n, n, 2, tau=taus, storage="f32", reaction="gray_scott", **kw))
    assert s.tuning().fused_steps >= 2          # the benchmark's multi-step launches
    s.init(rho0)
    f64 = oracle.init(rho0)
    f32 = oracle.init(rho0, "f32")
    done = 0
    t0 = time.time()
    for cp in (1000, 5000, 20000):
        s.step(cp - done)
        while done < cp:       # the oracle in chunks, reporting progress
            n = min(1000, cp - done)
            f64 = oracle.run(f64, n, taus, oracle.REACT_GRAY_SCOTT, **kw)
            f32 = oracle.run(f32, n, taus, oracle.REACT_GRAY_SCOTT, **kw)
            done += n
            print(f"oracle at step {done}, {time.time() - t0:.0f} s", flush=True)
        ref = oracle.moments(f64)
        floor = oracle.rel_l2(oracle.moments(f32), ref)
        rho, mass = s.moments()
        err = oracle.rel_l2(rho.cpu().numpy(), ref)
        tol = np.where(floor <= 1e-6, 1e-5, 3 * floor)
        print(f"GS f32 1024^2 step {cp}: rel L2 {err}, FP32 floor {floor}, tolerance {tol}, "
              f"mass rel diff {np.abs(mass - oracle.mass(ref)) / oracle.mass(ref)}, "
              f"{time.time() - t0:.0f} s", flush=True)
        assert np.all(err <= tol), (cp, err, floor)
    assert s.time() == 20000
