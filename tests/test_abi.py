"""Host-side checks of the C ABI (no GPU needed)."""
import ctypes as C
import os

import pytest

from paper_2405_13973_amd import native


def test_library_exports_every_declared_symbol():
    lib = native.load()
    names = native.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_header_declares_status_codes():
    txt = open(native.HEADER).read()
    for code in ("PT_OK = 0", "PT_EINVAL = -1", "PT_ENOMEM = -2", "PT_EDEVICE = -3", "PT_ENUMERIC = -4",
                 "PT_EBUSY = -5"):
        assert code in txt


def test_null_arguments_are_rejected_without_a_device():
    lib = native.load()
    assert lib.pt_ctx_create(0, 0, None, None) == native.PT_EINVAL
    assert lib.pt_ctx_destroy(None) == native.PT_EINVAL
    assert lib.pt_step(None, 1) == native.PT_EINVAL
    assert lib.pt_read_state(None, None, None, None, None, None) == native.PT_EINVAL
    assert lib.pt_compute_forces(None, None) == native.PT_EINVAL
    assert b"NULL" in lib.pt_last_error() or len(lib.pt_last_error()) > 0


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is visible here")
def test_ctx_create_without_device_fails_cleanly():
    lib = native.load()
    h = C.c_void_p()
    assert lib.pt_ctx_create(0, 0, None, C.byref(h)) == native.PT_EDEVICE
    assert not h.value


def test_numeric_status_reaches_the_caller():
    """PT_ENUMERIC (a step produced a non-finite state, reported at the next
    synchronising call) and every other status surfaces as PTError with its code."""
    lib = native.load()
    assert lib.pt_synchronize(None) == native.PT_EINVAL
    for code, name in ((native.PT_ENUMERIC, "PT_ENUMERIC"), (native.PT_ENOMEM, "PT_ENOMEM"),
                       (native.PT_EDEVICE, "PT_EDEVICE")):
        with pytest.raises(native.PTError) as e:
            native._check(code)
        assert e.value.code == code and name in str(e.value)
    native._check(native.PT_OK)


def test_library_resolves_its_own_symbols():
    """Every function of the library's own namespace is defined in it (a
    declaration that drifted from its definition would leave an undefined
    symbol that only fails when the library is loaded and called)."""
    import shutil
    import subprocess

    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm is not available")
    out = subprocess.run([nm, "-D", "--undefined-only", native.LIB_PATH], capture_output=True, text=True, check=True)
    own = [line for line in out.stdout.splitlines() if "_ZN2pt" in line]
    assert not own, own
