"""The C-ABI library loads and exports every symbol include/helrm.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "helrm.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(helrm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("helrm_create", "helrm_load_eval_keys", "helrm_ntt", "helrm_intt", "helrm_automorph",
                 "helrm_keyswitch_hoisted", "helrm_ptxt_ct_matvec_diag", "helrm_rescale",
                 "helrm_lookup_packed", "helrm_plan_create", "helrm_footprint"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_2506_18150_amd import binding
    lib = binding.lib()
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(binding.EXPORTS) == set(declared_symbols())


def test_errors_without_gpu_work():
    from paper_2506_18150_amd import binding
    lib = binding.lib()
    h = ctypes.c_void_p()
    assert lib.helrm_create(None, ctypes.byref(h)) == -1
    assert b"NULL" in lib.helrm_last_error()
    assert lib.helrm_destroy(None) == 0
