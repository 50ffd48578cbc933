"""lb_diag_noalloc (the entry point for callers that cannot allocate) against
lb_diag, through the C ABI: two calls in a row, the second on a smaller grid,
periodic and walled grids, every output bit for bit."""
import numpy as np
import pytest

from paper_1109_6672_amd import lbddf, workloads as W

pytestmark = pytest.mark.gpu


def _both(p, fields, steps):
    import torch

    s = lbddf.Solver(p).init(*fields).step(steps)
    out = torch.full((6,), float("nan"), dtype=torch.float64, device=s.device)
    s.diag_noalloc(out)
    s.stream.synchronize()
    got = out.cpu().numpy()
    ref = s.diag(check=False)
    want = np.array([ref["mass"], ref["energy"], ref["jx"], ref["jy"], ref["bad"], ref["time"]], dtype=np.float64)
    s.close()
    return got, want


@pytest.mark.parametrize("kind", ["periodic", "cavity"])
def test_diag_noalloc_matches_lb_diag(gpu, kind):
    cases = []
    for n, steps in ((300, 40), (70, 10)):  # the second call on a smaller grid
        if kind == "periodic":
            p = W.periodic(n, n // 2 + 3)
            f = W.gaussian_fields(p, sigma=1e-3)
        else:
            p = W.cavity(n, 1e5, 1.2, 0.06, sutherland=True)
            f = W.conduction_fields(p)
        cases.append((p, f, steps))
    for p, f, steps in cases:
        print(f"[case] lb_diag_noalloc vs lb_diag, {kind} {p['nx']}x{p['ny']}, {steps} steps", flush=True)
        got, want = _both(p, f, steps)
        assert np.all(np.isfinite(got)), got
        assert got.tobytes() == want.tobytes(), (got, want)
