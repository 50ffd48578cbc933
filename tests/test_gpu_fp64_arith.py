"""The library built with the step's arithmetic in FP64 (liblbddf_fp64.so;
FP32 storage): parity against the oracle where the FP32 step meets the bar
as well, and on the gravity-driven cavity where only FP64 arithmetic does;
the packed server on the same library."""
import numpy as np
import pytest

from paper_1109_6672_amd import lbddf, workloads as W
from tests.gpu_common import TOL, rel_errors

pytestmark = pytest.mark.gpu


def _pair(p, f, steps):
    from oracle import oracle as O

    s = lbddf.Solver(p, arith="f64").init(*f).step(steps)
    o = O.Oracle(p).init(*f).step(steps)
    return s, o, rel_errors(s.macros(), o.macros())


def test_periodic_noise(gpu):
    p = W.periodic(150, 77)
    _, _, e = _pair(p, W.gaussian_fields(p, sigma=1e-3), 200)
    print(f"[case] FP64 arithmetic, periodic noise 150x77: {e}", flush=True)
    assert max(e) < TOL["f32"], e


def test_small_dT_cavity_long_horizon(gpu):
    """70 x 70 small-dT cavity after 12,000 steps: FP32 arithmetic is 3.8e-4
    off in u here, FP64 arithmetic with FP32 storage 8e-7."""
    p = W.cavity(70, 1e4, 0.02, 0.02)
    _, _, e = _pair(p, W.noisy_temperature_fields(p), 12_000)
    print(f"[case] FP64 arithmetic, cavity 70x70, 12000 steps: {e}", flush=True)
    assert max(e) < TOL["f32"], e


def test_channel_inlet_outlet(gpu):
    p = W.channel(nx=190, ny=9, U0=0.01, period=40.0)
    _, _, e = _pair(p, W.rest_fields(p), 600)
    assert max(e) < TOL["f32"], e


def test_server_on_the_fp64_library(gpu):
    from oracle import oracle as O

    p = W.cavity(70, 1e4, 0.02, 0.02)
    f = W.noisy_temperature_fields(p)
    srv = lbddf.Server(lbddf.load("f64").lbs_pool_overhead() + lbddf.state_bytes(p) + 256, k_steps=100,
                       arith="f64")
    rid = srv.submit(p, f, tol=0.0, max_steps=2000)
    for _ in range(100):
        r, q = srv.advance()
        if r == 0 and q == 0:
            break
    e = rel_errors(srv.result(rid), O.Oracle(p).init(*f).step(2000).macros())
    print(f"[case] FP64 arithmetic server, cavity 70x70, 2000 steps: {e}", flush=True)
    assert max(e) < TOL["f32"], e
