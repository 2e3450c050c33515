"""The C-ABI library loads and exports every entry point include/bem.h declares,
and rejects bad arguments before touching a device (runs without a GPU)."""
import ctypes

import pytest

from paper_2602_05492_amd import bem as B


def test_header_lists_the_hot_path_calls():
    names = B.header_functions()
    for n in ("bem_build", "bem_factor", "bem_eval", "bem_vjp", "bem_jtj", "lm_step", "bem_jacobian",
              "bem_destroy", "bem_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in B.header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(B.header_functions()) == set(B._SIGS)


def _opts(**kw):
    o = dict(elems_per_side=256, segs_per_handle=32, eps=1e-2, near_factor=1.0, tile_rows=0, device=0,
             handle_model=0)
    o.update(kw)
    return B.Opts(**o)


@pytest.mark.parametrize("bad", [dict(elems_per_side=1), dict(elems_per_side=5000), dict(segs_per_handle=0),
                                 dict(eps=-1.0), dict(eps=float("nan")), dict(near_factor=0.0),
                                 dict(tile_rows=-3), dict(handle_model=2), dict(handle_model=-1)])
def test_build_rejects_bad_options(bad):
    L = B.lib()
    h = ctypes.c_void_p()
    rc = L.bem_build(ctypes.byref(_opts(**bad)), None, ctypes.byref(h))
    assert rc == -1
    assert h.value is None
    assert L.bem_last_error(None)


def test_opts_struct_matches_header():
    """bem_opts: the binding's field order and sizes are the header's."""
    src = open(B.HEADER).read()
    body = src[src.index("typedef struct {\n    int32_t elems_per_side"):]
    body = body[:body.index("} bem_opts;")]
    fields = [ln.split(";")[0].split()[-1] for ln in body.splitlines()[1:] if ";" in ln]
    assert fields == [f[0] for f in B.Opts._fields_]


def test_null_arguments():
    L = B.lib()
    assert L.bem_build(None, None, None) == -1
    assert L.bem_factor(None, None) == -1
    cb = (ctypes.c_double * 3)(0, 0, 0)
    assert L.bem_eval(None, None, 0, None, 0, cb, None, 0, None) == -1
    assert L.bem_num_elements(None) == 0
    assert L.bem_near_capacity(None) == 0
    assert L.bem_set_regularization(None, None) == -1
    v, k = ctypes.c_double(), ctypes.c_int32()
    assert L.bem_regularization(None, None, 0, ctypes.byref(v), None, None, None, None) == -1
    assert L.bem_prune(None, None, 0, 0.0, ctypes.byref(k), None) == -1
    L.bem_destroy(None)
