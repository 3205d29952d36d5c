"""Context memory through the caller's allocator (cav_create's cav_allocator).

With the binding's default allocator (PyTorch's caching allocator) a setup and
a solve must take every device block from the hook (no hipMalloc of the
library's own), torch must account for that memory while the context lives,
and every block must be returned when the context closes. Without an
allocator the library allocates for itself. Both give the same solve bit for
bit (same kernels, same inputs).
"""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _run(allocator):
    from paper_2608_14310_amd import Solver
    s = workloads.membrane_ellipse(64, 4, 1e4, 1)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    g = Solver(0, allocator=allocator)
    hook = g.allocator
    g.setup(s, alpha=1.0, smoother="multiplicative")
    b = torch.from_numpy(s.b).cuda()
    x, info = g.fgmres_solve(b, rtol=1e-10, max_it=150)
    torch.cuda.synchronize()
    mem = g.memory_stats()
    held = torch.cuda.memory_allocated() - base
    hook_live = hook.live_bytes if hook is not None else 0
    out = x.cpu().numpy()
    g.close()
    torch.cuda.synchronize()
    return dict(x=out, info=info, mem=mem, held=held, hook=hook, hook_live=hook_live, base=base,
                after=torch.cuda.memory_allocated())


def test_setup_and_solve_allocate_only_through_the_hook():
    r = _run("torch")
    m, hook = r["mem"], r["hook"]
    print(f"[memory] torch hook: {m}, torch-held {r['held']} bytes", flush=True)
    assert r["info"]["converged"] == 1
    assert m["hip_malloc_calls"] == 0
    assert m["allocator_allocs"] == hook.allocs > 0
    # blocks in use plus blocks the context keeps for reuse: all from the hook
    assert m["live_bytes"] + m["cached_bytes"] == r["hook_live"] > 0
    # the context's memory is torch memory while the context lives
    assert r["held"] >= m["live_bytes"] + m["cached_bytes"]
    # and all of it went back on close
    assert hook.frees == hook.allocs and hook.live_bytes == 0
    # (torch accounts each block at its own rounding, at least the requested size)
    assert r["after"] <= r["base"] + r["held"] - m["live_bytes"] - m["cached_bytes"]


def test_without_allocator_the_library_allocates_and_results_agree():
    a = _run("torch")
    b = _run(None)
    print(f"[memory] no hook: {b['mem']}", flush=True)
    assert b["mem"]["allocator_allocs"] == 0 and b["mem"]["hip_malloc_calls"] > 0
    assert a["info"]["iterations"] == b["info"]["iterations"]
    assert np.array_equal(a["x"], b["x"])
