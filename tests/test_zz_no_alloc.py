"""The allocation-free CCD bound (ipc_ccd_bound_pairs_noalloc) against the allocating entry point
(ipc_ccd_bound_pairs) through the C-ABI: two calls in a row on the same GPU, the second with fewer
pairs (the shared per-block minima of the first call must not leak into the second), each equal bit
for bit to the allocating call on the same pairs (same kernels, exact minima); sizes beyond the fixed
scratch are rejected before anything is queued.

The caller's device buffers are allocated here with hipMalloc of the HIP runtime the library itself
is linked against (found among the loaded libraries), so the test needs no other GPU framework."""
import ctypes as C

import numpy as np
import pytest

from paper_2503_05020_amd import ipc as G

pytestmark = pytest.mark.gpu


def _hip():
    """The libamdhip64 the IPC library loaded (same runtime, same device memory)."""
    G.lib()
    with open("/proc/self/maps") as f:
        paths = {ln.split()[-1] for ln in f if "libamdhip64.so" in ln}
    own = [p for p in paths if p.startswith("/opt/rocm")] or sorted(paths)
    hip = C.CDLL(own[0])
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipFree.argtypes = [C.c_void_p]
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    hip.hipDeviceSynchronize.argtypes = []
    return hip


H2D, D2H = 1, 2


class DevBuf:
    def __init__(self, hip, nbytes):
        self.hip = hip
        self.p = C.c_void_p()
        assert hip.hipMalloc(C.byref(self.p), max(8, nbytes)) == 0

    def put(self, a):
        a = np.ascontiguousarray(a)
        assert self.hip.hipMemcpy(self.p, a.ctypes.data, a.nbytes, H2D) == 0

    def get(self, n):
        out = np.zeros(n)
        assert self.hip.hipMemcpy(out.ctypes.data, self.p, out.nbytes, D2H) == 0
        return out

    def free(self):
        self.hip.hipFree(self.p)


def _pairs(rng, n):
    return rng.uniform(-1, 1, (n, 12)), rng.uniform(-0.3, 0.3, (n, 12))


@pytest.mark.parametrize("kind", [0, 1])
def test_noalloc_ccd_bound_matches_allocating_call(kind):
    hip = _hip()
    rng = np.random.default_rng(5 + kind)
    # first call: many pairs over many blocks; second: fewer pairs in fewer blocks
    results = []
    for n in (20000, 300):
        x, p = _pairs(rng, n)
        xd, pd, ad = DevBuf(hip, x.nbytes), DevBuf(hip, p.nbytes), DevBuf(hip, 8)
        xd.put(x)
        pd.put(p)
        ad.put(np.array([-1.0]))
        print(f"kind {kind}: noalloc call with {n} pairs", flush=True)
        G.ipc_ccd_bound_pairs_noalloc(kind, n, xd.p.value, pd.p.value, ad.p.value, 0.1, None)
        assert hip.hipDeviceSynchronize() == 0
        got = float(ad.get(1)[0])
        ref = G.ipc_ccd_bound_pairs(kind, x, p)
        print(f"  noalloc {got:.17g} allocating {ref:.17g}", flush=True)
        for b in (xd, pd, ad):
            b.free()
        assert got == ref
        assert 0.0 < got <= 1.0
        results.append(got)
    # both lists bind (the bound is below 1), so a stale partial would have shown as a difference
    assert max(results) < 1.0


def test_noalloc_rejects_oversized_and_bad_arguments():
    hip = _hip()
    buf, a = DevBuf(hip, 24 * 8), DevBuf(hip, 8)
    lib = G.lib()
    too_many = (1 << 16) * 128 + 1
    rc = lib.ipc_ccd_bound_pairs_noalloc(0, too_many, buf.p.value, buf.p.value, 0.1, a.p.value, None)
    assert rc == G.IPC_E_ARG
    assert "scratch" in G.ipc_last_error()
    assert lib.ipc_ccd_bound_pairs_noalloc(2, 1, buf.p.value, buf.p.value, 0.1, a.p.value, None) == G.IPC_E_ARG
    assert lib.ipc_ccd_bound_pairs_noalloc(0, 1, buf.p.value, buf.p.value, 1.5, a.p.value, None) == G.IPC_E_ARG
    # an empty list gives 1
    a.put(np.array([-1.0]))
    assert lib.ipc_ccd_bound_pairs_noalloc(1, 0, None, None, 0.1, a.p.value, None) == G.IPC_OK
    assert hip.hipDeviceSynchronize() == 0
    assert float(a.get(1)[0]) == 1.0
    buf.free()
    a.free()
