"""The allocation-free entry point (pma_solve_subdomain_noalloc) against pma_solve_subdomain.

Both advance one subdomain in place on a caller-owned device buffer; the allocation-free one
keeps its state, DCT matrices and launch tables in the library's fixed device scratch and
launches on the caller's stream directly.  Same kernels and tiles, so the results must be
bitwise equal; both are also checked against the FP64 oracle (1e-11 FP64, 2e-6 FP32 forms, as
the Dirichlet-subdomain parity test).  Two calls in a row, the second on a smaller subdomain
(the scratch keeps the first call's contents), and no device memory taken through torch.
"""
import numpy as np
import pytest

import oracle as O
from paper_2006_14602_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 2e-6, "split16": 2e-6}


def _case(n, lo, hi, faces, steps, seed):
    # subdomain [lo, hi] of a grid with n nodes per axis; faces: (low artificial, high artificial)
    # per axis; Dirichlet data = a perturbed Psi held fixed on artificial faces
    d = len(n)
    g = W.grid(list(n))
    gs = O.GridSpec(tuple(n), (0.0,) * d, (1.0,) * d)
    box = O.Box(tuple(lo), tuple(h - l + 1 for l, h in zip(lo, hi)), gs.h, gs.lo, gs.hi,
                tuple(bool(f[0]) for f in faces), tuple(bool(f[1]) for f in faces))
    X = box.coords()
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 1.5, d)
    psi0 = 0.5 * np.sum(X * X, -1) + 1e-3 * np.prod([np.cos(np.pi * a[k] * X[..., k]) for k in range(d)], 0)
    mon = W.ring_monitor(d=d)
    t = {"dt": 1e-3, "gamma": 1.0, "steps": steps}
    th = O.theta(mon, gs.lo, gs.hi)
    p = psi0.copy()
    for _ in range(steps):
        p, _ = O.step_box(p, box, mon, th, gs.vol, t["dt"], t["gamma"])
    fk = [v for f in faces for v in f]
    return g, lo, hi, fk, mon, t, psi0, p


CASES = [  # larger first, then smaller
    ((97, 81), (20, 0), (96, 60), ((1, 0), (0, 1)), 30, 1),
    ((49, 33), (10, 0), (40, 32), ((1, 1), (0, 0)), 20, 2),
]
CASES3 = [
    ((41, 37, 33), (0, 4, 0), (40, 36, 20), ((0, 0), (1, 0), (0, 1)), 12, 3),
    ((25, 21, 19), (3, 0, 0), (20, 20, 18), ((1, 1), (0, 0), (0, 0)), 10, 4),
]


@pytest.mark.parametrize("cases", [CASES, CASES3], ids=["2d", "3d"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "split16"])
def test_noalloc_equals_solve_subdomain(lib, cases, prec):
    import torch
    from paper_2006_14602_amd import binding
    with binding.Context(0, budget_bytes=256 << 20) as ctx:
        for (n, lo, hi, faces, steps, seed) in cases:
            g, lo, hi, fk, mon, t, psi0, ref = _case(n, lo, hi, faces, steps, seed)
            print(f"case noalloc {prec} n={n} lo={lo} hi={hi}", flush=True)
            a = torch.tensor(psi0, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            m0 = torch.cuda.memory_allocated()
            sa = ctx.solve_subdomain(g, lo, hi, fk, mon, t, a, precision=prec, noalloc=True)
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated() == m0   # nothing taken through torch's allocator
            b = torch.tensor(psi0, dtype=torch.float64, device="cuda")
            sb = ctx.solve_subdomain(g, lo, hi, fk, mon, t, b, precision=prec)
            A, Bv = a.cpu().numpy(), b.cpu().numpy()
            np.testing.assert_array_equal(A, Bv)
            assert sa["steps_done"] == sb["steps_done"] == steps
            err = float(np.max(np.abs(A - ref)))
            print(f"noalloc {prec} n={n}: max |Psi - oracle| {err:.3e}", flush=True)
            assert err <= TOL[prec]


def test_noalloc_rejects_oversize(lib):
    import torch
    from paper_2006_14602_amd import binding
    g = W.grid([150, 150, 150])
    mon = W.ring_monitor(d=3)
    t = {"dt": 1e-3, "gamma": 1.0, "steps": 1}
    psi = torch.zeros((150, 150, 150), dtype=torch.float64, device="cuda")
    with binding.Context(0, budget_bytes=256 << 20) as ctx:
        with pytest.raises(binding.PmaError) as e:
            ctx.solve_subdomain(g, [0, 0, 0], [149, 149, 149], [0] * 6, mon, t, psi, precision="fp64", noalloc=True)
        assert e.value.code == binding.PMA_E_INVAL
        assert "allocation-free" in str(e.value)
