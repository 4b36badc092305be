"""The C ABI: the built library loads and exports every function that
include/*.h declares; the Python binding names them all.  No GPU calls are
made (host-only entry points only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]
LIB = os.path.join(ROOT, "paper_2212_09664_amd", "libaltgdmin.so")


def declared():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:altgdmin|wsinit)_[a-z_A-Z0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared()
    for must in ("altgdmin_init", "altgdmin_iterate", "altgdmin_apply_A", "altgdmin_apply_AH",
                 "altgdmin_create", "altgdmin_set_problem", "altgdmin_destroy", "altgdmin_cnn_input",
                 "altgdmin_init_warm", "altgdmin_init_warm_from", "wsinit_create", "wsinit_forward", "wsinit_loss_backward",
                 "wsinit_adam_step"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_every_declared_symbol():
    from paper_2212_09664_amd import _lib
    src = open(_lib.__file__).read()
    missing = [n for n in declared() if f'"{n}"' not in src]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_only_argument_checks():
    """altgdmin_create validates shapes on the host without touching a GPU."""
    from paper_2212_09664_amd import _lib
    L = _lib.load_library()
    P = _lib.Params
    h = ctypes.c_void_p()
    ok = P(64, 64, 4, 16, 4, 1024, 0, 0, 36.0, 0.14, 0.0, 0.0, 70)
    assert L.altgdmin_create(ctypes.byref(ok), ctypes.byref(h)) == 0
    nb = ctypes.c_size_t()
    assert L.altgdmin_workspace_bytes(h, ctypes.byref(nb)) == 0 and nb.value > 0
    L.altgdmin_destroy(h)
    for bad in (P(48, 64, 4, 16, 4, 1024, 0, 0, 36.0, 0.14, 0.0, 0.0, 70),   # nx not 2^k
                P(64, 64, 4, 16, 17, 1024, 0, 0, 36.0, 0.14, 0.0, 0.0, 70),  # r > 16
                P(64, 64, 4, 16, 4, 1024, 0, 0, 36.0, 0.14, 0.0, 0.0, 70, -1),  # exit_consec < 0
                P(64, 64, 4, 16, 4, 1000, 0, 0, 36.0, 0.14, 0.0, 0.0, 70),   # m_max % nx
                P(64, 64, 4, 16, 4, 1024, 2, 0, 36.0, 0.14, 0.0, 0.0, 70),   # mask kind
                P(64, 64, 4, 16, 4, 1024, 0, 0, 36.0, 0.0, 0.0, 0.0, 70)):   # eta_c
        assert L.altgdmin_create(ctypes.byref(bad), ctypes.byref(h)) == 1
    assert L.altgdmin_status_string(4) == b"Gram matrix not positive definite"
    # r > q is a valid context (LS step, operators, the steps around the loop);
    # the spectral initialisation refuses it
    wide = P(64, 64, 4, 1, 4, 1024, 0, 0, 36.0, 0.14, 0.0, 0.0, 70)
    assert L.altgdmin_create(ctypes.byref(wide), ctypes.byref(h)) == 0
    assert L.altgdmin_init(h, ctypes.c_void_p(256)) == 1
    nb = ctypes.c_size_t()
    assert L.altgdmin_aux_bytes(h, ctypes.byref(nb)) == 0 and nb.value > 0
    # the steps around the loop check their arguments before any launch
    one = ctypes.c_void_p(256)
    assert L.altgdmin_mean(h, -1.0, 10, one, one, None) == 1          # tol < 0
    assert L.altgdmin_mean(h, 1e-3, 10, one, ctypes.c_void_p(300), None) == 1  # unaligned aux
    assert L.altgdmin_mec_cgls(h, one, -1, 0.0, one, one) == 1        # iters < 0
    assert L.altgdmin_mec_ista(h, one, 10, -1.0, 0.0, one, one, None) == 1
    assert L.altgdmin_rank_energy(h, 17, (ctypes.c_double * 17)(), one) == 1
    assert L.altgdmin_expand(h, one, None, None, None, one) == 1       # U without B
    assert L.altgdmin_mean(h, 1e-3, 10, one, one, None) == 2           # no problem bound yet
    L.altgdmin_destroy(h)
    # the no-allocation mean refuses, before anything else, a problem whose
    # scratch (8 (3 + nc) n bytes) exceeds its built-in 16 MiB
    big = P(512, 512, 8, 4, 2, 512 * 8, 0, 0, 36.0, 0.14, 0.0, 0.0, 70)
    assert L.altgdmin_create(ctypes.byref(big), ctypes.byref(h)) == 0
    assert L.altgdmin_mean_noalloc(h, 1e-3, 10, one, None) == 7
    L.altgdmin_destroy(h)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_wsinit_host_checks_and_parameter_count():
    from paper_2212_09664_amd import _lib
    L = _lib.load_library()
    h = ctypes.c_void_p()
    assert L.wsinit_create(128, 128, 48, 6, 32, 4, 4, None, ctypes.byref(h)) == 0
    c = ctypes.c_int64()
    assert L.wsinit_param_count(h, ctypes.byref(c)) == 0 and c.value == 49644
    nb = ctypes.c_size_t()
    assert L.wsinit_workspace_bytes(h, ctypes.byref(nb)) == 0 and nb.value > 0
    L.wsinit_destroy(h)
    for bad in ((100, 128, 48, 6, 32, 4, 4), (128, 128, 48, 17, 32, 4, 4), (128, 128, 48, 6, 33, 4, 4),
                (128, 128, 48, 6, 32, 3, 4), (128, 128, 48, 6, 32, 4, 0), (128, 128, 129, 6, 32, 4, 4)):
        h = ctypes.c_void_p()
        assert L.wsinit_create(*bad, None, ctypes.byref(h)) == 1, bad
