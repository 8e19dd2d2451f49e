"""The allocation-free entry point bscf_guess_eval_noalloc against
bscf_guess_eval, the entry point it is a variant of: the same network output
for device rows, on two calls in a row (the second with fewer rows, so it
reuses the per-GPU activation array left as the first call wrote it), and a
refusal of more rows than the array holds.

Device buffers for the caller's inputs and outputs come from the HIP runtime
that libbeadscf.so itself is linked against (through ctypes), so no second
HIP runtime enters the process."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _hip_runtime():
    """The libamdhip64 that the loaded libbeadscf.so uses (same handle)."""
    from paper_1601_02713_amd import beadscf  # noqa: F401  (loads the library)
    with open("/proc/self/maps") as f:
        paths = sorted({ln.split()[-1] for ln in f if "libamdhip64.so" in ln})
    assert len(paths) == 1, paths
    hip = ctypes.CDLL(paths[0])
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    for fn in (hip.hipMalloc, hip.hipFree, hip.hipMemcpy, hip.hipDeviceSynchronize):
        fn.restype = ctypes.c_int
    return hip


class _DevBuf:
    H2D, D2H = 1, 2

    def __init__(self, hip, nbytes):
        self.hip, self.p = hip, ctypes.c_void_p()
        assert hip.hipMalloc(ctypes.byref(self.p), nbytes) == 0
        self.nbytes = nbytes

    def put(self, a):
        a = np.ascontiguousarray(a)
        assert a.nbytes <= self.nbytes
        assert self.hip.hipMemcpy(self.p, a.ctypes.data_as(ctypes.c_void_p), a.nbytes, self.H2D) == 0

    def get(self, shape, dtype):
        out = np.empty(shape, dtype)
        assert out.nbytes <= self.nbytes
        assert self.hip.hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), self.p, out.nbytes, self.D2H) == 0
        return out

    def free(self):
        if self.p:
            self.hip.hipFree(self.p)
            self.p = ctypes.c_void_p()


def test_noalloc_eval_matches_eval_on_two_calls():
    from paper_1601_02713_amd import beadscf
    from oracle import mlp
    hip = _hip_runtime()
    e = beadscf.Engine(0)
    bufs = []
    try:
        din, dout = 70, 9
        e.guess_configure(din, dout)
        rng = np.random.default_rng([2000, 77])
        th = mlp.init(din, 256, dout, rng)
        W1, b1, W2, b2, W3, b3 = mlp.unflatten(th, din, 256, dout)
        th = mlp.flatten([W1, rng.standard_normal(b1.shape) * 0.1, W2,
                          rng.standard_normal(b2.shape) * 0.1,
                          rng.standard_normal(W3.shape) * 0.06,
                          rng.standard_normal(b3.shape) * 0.1]).astype(np.float32)
        e.guess_set_params(th)
        xd = _DevBuf(hip, 5000 * din * 4)
        yd = _DevBuf(hip, 5000 * dout * 4)
        bufs += [xd, yd]
        for rows in (5000, 777):
            X = rng.standard_normal((rows, din)).astype(np.float32)
            Y_ref, _, _ = e.guess_eval(X)
            xd.put(X)
            yd.put(np.full((rows, dout), np.nan, np.float32))
            e.guess_eval_noalloc(rows, xd.p.value, yd.p.value)
            assert hip.hipDeviceSynchronize() == 0
            Y = yd.get((rows, dout), np.float32)
            assert np.isfinite(Y).all()
            assert np.abs(Y - Y_ref).max() <= 1e-6 * np.abs(Y_ref).max(), rows
        with pytest.raises(beadscf.BscfError) as ei:
            e.guess_eval_noalloc(8193, xd.p.value, yd.p.value)
        assert ei.value.code == -1 and "8192" in str(ei.value)
    finally:
        for b in bufs:
            b.free()
        e.close()
