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


def _header_struct(name):
    """(field name, C type) of the typedef'd struct `name` in the header, in order."""
    src = open(B.HEADER).read()
    end = src.index("} %s;" % name)
    body = src[src.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    out = []
    for ln in body.splitlines():
        decl = ln.split("/*")[0].strip()
        if not decl.endswith(";"):
            continue
        parts = decl[:-1].split()
        out.append((parts[-1].split("[")[0], parts[0], "[" in parts[-1]))
    return out


_CTYPES = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double}


@pytest.mark.parametrize("name,cls", [("bem_opts", "Opts"), ("bem_lm_state", "LMState"), ("bem_reg", "Reg")])
def test_structs_match_header(name, cls):
    """The binding's ctypes structs have the header's fields, in order, with the same C types."""
    fields = _header_struct(name)
    ct = getattr(B, cls)._fields_
    alias = {"lambda": "lam"}                      # a Python keyword
    assert [alias.get(f[0], f[0]) for f in fields] == [f[0] for f in ct]
    for (fname, ctype, is_arr), (_, cty) in zip(fields, ct):
        base = cty._type_ if is_arr else cty
        assert base is _CTYPES[ctype], (fname, ctype, cty)


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
