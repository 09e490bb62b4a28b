"""gnk_cauchy_sum_noalloc (the Cauchy sum that allocates nothing: its workspace
is the library's fixed per-GPU scratch array) through the C ABI, against
gnk_cauchy_sum on the same inputs: two calls in a row, the second smaller, an
input too large for the scratch (rejected, output untouched), and a call after
it."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gk():
    from paper_1308_5351_amd import gnk
    assert torch.cuda.is_available()
    return gnk


def _inputs(N, nrhs, seed):
    """N nodes on the 17-component boundary's first N nodes (distinct points) and
    seeded complex weights, as complex128 CUDA tensors."""
    dom, _ = wl.config1()
    eta = dom.eta
    if N > eta.shape[0]:
        dom4, _ = wl.config4()
        eta = dom4.eta
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(nrhs, N)) + 1j * rng.normal(size=(nrhs, N))
    return (torch.from_numpy(np.ascontiguousarray(eta[:N])).cuda(),
            torch.from_numpy(np.ascontiguousarray(w)).cuda())


def _sum(ctx, fn, eta, w):
    nrhs, N = w.shape
    S = torch.full_like(w, complex(float("nan"), float("nan")))
    st = fn(ctx.h, N, eta.data_ptr(), w.data_ptr(), nrhs, S.data_ptr())
    torch.cuda.synchronize()
    return st, S


@pytest.mark.parametrize("shapes", [((16384, 2), (3001, 1)), ((4096, 8), (1000, 3)), ((65536, 1), (2048, 2))])
def test_noalloc_matches_allocating_entry_point(gk, shapes):
    ctx = gk.Context(0)
    lib = ctx.lib
    try:
        for k, (N, nrhs) in enumerate(shapes):
            print(f"[noalloc] call {k}: N={N} nrhs={nrhs}", flush=True)
            eta, w = _inputs(N, nrhs, [N, nrhs])
            st_a, S_a = _sum(ctx, lib.gnk_cauchy_sum, eta, w)
            st_n, S_n = _sum(ctx, lib.gnk_cauchy_sum_noalloc, eta, w)
            assert st_a == 0 and st_n == 0, lib.gnk_last_error(ctx.h)
            err = float((S_n - S_a).abs().max() / S_a.abs().max())
            print(f"  max rel diff {err:.2e}, bitwise equal {bool(torch.equal(S_n, S_a))}", flush=True)
            assert torch.isfinite(S_n).all() and err <= 1e-14
    finally:
        ctx.close()


def test_noalloc_rejects_inputs_beyond_its_scratch(gk):
    ctx = gk.Context(0)
    lib = ctx.lib
    try:
        eta, w = _inputs(264192, 1, 5)
        print("[noalloc] oversize N=264192", flush=True)
        st, S = _sum(ctx, lib.gnk_cauchy_sum_noalloc, eta, w)
        msg = lib.gnk_last_error(ctx.h).decode()
        print(f"  status {st}: {msg}", flush=True)
        assert st == gk.ERR_ARG and "scratch" in msg
        assert torch.isnan(S.real).all()                  # nothing written
        eta, w = _inputs(2048, 2, 6)                       # and the next call works
        st_a, S_a = _sum(ctx, lib.gnk_cauchy_sum, eta, w)
        st_n, S_n = _sum(ctx, lib.gnk_cauchy_sum_noalloc, eta, w)
        assert st_a == 0 and st_n == 0
        assert float((S_n - S_a).abs().max() / S_a.abs().max()) <= 1e-14
    finally:
        ctx.close()


def test_noalloc_takes_no_device_memory(gk):
    """A fresh context's first no-alloc call leaves the free device memory as it
    was (the allocating entry point grows a workspace of tens of MB for the same
    input)."""
    eta, w = _inputs(16384, 2, 7)
    torch.cuda.synchronize()
    ctx = gk.Context(0)
    try:
        free0, _ = torch.cuda.mem_get_info()
        st, _ = _sum(ctx, ctx.lib.gnk_cauchy_sum_noalloc, eta, w)
        free1, _ = torch.cuda.mem_get_info()
        st_a, _ = _sum(ctx, ctx.lib.gnk_cauchy_sum, eta, w)
        free2, _ = torch.cuda.mem_get_info()
        print(f"[noalloc] free memory change: no-alloc {free0 - free1} B, allocating {free1 - free2} B", flush=True)
        assert st == 0 and st_a == 0
        assert free0 - free1 < (16 << 20)
    finally:
        ctx.close()
