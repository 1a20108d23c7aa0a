"""Context life cycle on the GPU: repeated pma_create / pma_destroy with solves, plans and served
requests in between leave no device memory, host memory or threads behind.

Each cycle creates a context (arena from hipMalloc, or from torch's caching allocator through the
allocation callbacks), runs a batched FP64 solve, a split-form decomposed solve, a plan and two
served requests (which start the server thread), and destroys the context.  After a warm-up cycle
of each kind (first-use allocations of the HIP runtime), eight more cycles must return:
  - device memory outside torch's cache (hipMemGetInfo) to within 8 MiB,
  - bytes held through torch's allocator exactly,
  - the process's thread count to within 3 (a server thread left running per cycle would add 8),
  - the resident host memory to within 64 MiB.
"""
import os
import time

import pytest

from paper_2006_14602_amd import workloads as W

pytestmark = pytest.mark.gpu


def _threads():
    return len(os.listdir("/proc/self/task"))


def _cycle(binding, use_torch):
    ring = W.ring(steps=20)
    ring["grid"] = W.grid([49, 49])
    dd = W.sine_dd(n=65, parts=(2, 2), overlap=4, steps=20)
    with binding.Context(0, budget_bytes=256 << 20, use_torch_allocator=use_torch) as c:
        c.dd_mesh(ring, precision="fp64")
        c.dd_mesh(dd, precision="split16")
        with binding.Plan(c, [ring, dd], "fp64", "batched") as p:
            p.step(10)
            p.sync()
        tickets = [c.submit(ring, "split16"), c.submit(dd, "fp64")]
        shapes = [(2, 49, 49), (2, 65, 65)]
        t0 = time.time()
        done = set()
        while len(done) < 2:
            for i, t in enumerate(tickets):
                if i not in done and c.poll(t, shape=shapes[i])[0] in (2, 3):
                    done.add(i)
            assert time.time() - t0 < 60, "serving did not finish"
            time.sleep(0.002)


def test_create_destroy_releases_everything(lib):
    import psutil
    import torch
    from paper_2006_14602_amd import binding
    _cycle(binding, False)
    _cycle(binding, True)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0] + torch.cuda.memory_reserved(0)
    held0 = torch.cuda.memory_allocated(0)
    th0 = _threads()
    rss0 = psutil.Process().memory_info().rss
    for i in range(8):
        _cycle(binding, i % 2 == 0)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info(0)[0] + torch.cuda.memory_reserved(0)
    held1 = torch.cuda.memory_allocated(0)
    th1 = _threads()
    rss1 = psutil.Process().memory_info().rss
    print(f"device free (incl. torch cache) {free0 / 2**20:.1f} -> {free1 / 2**20:.1f} MiB, "
          f"torch-held {held0} -> {held1} B, threads {th0} -> {th1}, rss {rss0 / 2**20:.1f} -> {rss1 / 2**20:.1f} MiB")
    assert free0 - free1 < 8 << 20
    assert held1 == held0
    assert th1 - th0 < 4
    assert rss1 - rss0 < 64 << 20
