"""The force entry point that allocates nothing (pt_compute_forces_noalloc)
against the allocating one (pt_compute_forces, direct method): bit for bit, on
two calls in a row -- the first at the size limit, the second with a smaller
crystal, so the second call runs on scratch the first one left dirty -- with
the context's device memory unchanged by either call; and its limits.

The caller's device buffers come from the HIP runtime the library itself is
linked against (libamdhip64 through ctypes), so the test holds no second
runtime."""
import ctypes as C

import numpy as np
import pytest

from paper_2405_13973_amd import inputs, native

pytestmark = pytest.mark.gpu

Q, M = inputs.ION_CHARGE, inputs.ION_MASS
N_MAX = 131072  # PT_NOALLOC_MAX_IONS


class DeviceBuffer:
    """n x 3 doubles of device memory, filled with NaN."""

    def __init__(self, n):
        native.load()  # the library, and with it its HIP runtime, first
        self.hip = C.CDLL("libamdhip64.so.7")
        self.n = n
        self.ptr = C.c_void_p()
        assert self.hip.hipMalloc(C.byref(self.ptr), C.c_size_t(24 * n)) == 0
        nan = np.full((n, 3), np.nan)
        assert self.hip.hipMemcpy(self.ptr, nan.ctypes.data_as(C.c_void_p), C.c_size_t(24 * n), 1) == 0

    def read(self):
        out = np.zeros((self.n, 3))
        assert self.hip.hipMemcpy(out.ctypes.data_as(C.c_void_p), self.ptr, C.c_size_t(24 * self.n), 2) == 0
        return out

    def free(self):
        assert self.hip.hipFree(self.ptr) == 0


def test_noalloc_forces_equal_the_allocating_entry_point():
    with native.Context(0) as ctx:
        for n, seed in ((N_MAX, 61), (3001, 62)):
            print(f"noalloc n={n}", flush=True)
            pos = inputs.uniform_ball(n, inputs.density_radius(n), inputs.rng(seed))
            c = ctx.crystal(pos, np.zeros_like(pos), Q, M, seed)
            c.set_force("direct")
            ref = c.compute_forces()
            F = DeviceBuffer(n)
            before = ctx.memory()[0]
            c.compute_forces_noalloc(F.ptr.value)
            ctx.synchronize()
            assert ctx.memory()[0] == before
            got = F.read()
            F.free()
            assert np.array_equal(got, ref)
            c.destroy()


def test_noalloc_limits():
    with native.Context(0) as ctx:
        F = DeviceBuffer(N_MAX + 1)
        pos = inputs.uniform_ball(N_MAX + 1, 1e-3, inputs.rng(63))
        c = ctx.crystal(pos, np.zeros_like(pos), Q, M, 63)
        c.set_force("direct")
        with pytest.raises(native.PTError) as e:
            c.compute_forces_noalloc(F.ptr.value)
        assert e.value.code == native.PT_EINVAL
        c.destroy()
        c = ctx.crystal(pos[:100], np.zeros((100, 3)), Q, M, 64)
        c.set_force("fmm", 8, 32)
        with pytest.raises(native.PTError) as e:
            c.compute_forces_noalloc(F.ptr.value)
        assert e.value.code == native.PT_EINVAL
        assert native.load().pt_compute_forces_noalloc(c.h, None) == native.PT_EINVAL
        c.destroy()
        F.free()
