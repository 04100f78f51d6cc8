"""The C-ABI library loads and exports every symbol include/fvim.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fvim.h")
LIB = os.path.join(ROOT, "paper_1811_11558_amd", "libfvim.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "for", "sizeof")))


def test_header_declares_the_operator_and_solver_calls():
    names = declared_functions()
    for n in ("mindlin_apply", "boussinesq_apply", "return_map", "contact_solve", "elastoplastic_solve",
              "tangential_solve", "fvim_set_depth_nodes"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_create_rejects_bad_grids_before_touching_a_device():
    from paper_1811_11558_amd import binding as b
    lib = b.load_library()
    m = b._Material(1.0, 0.3, 0.01, 0.1)
    h = ctypes.c_void_p()
    for g in (b._Grid(30, 32, 8, 1, 1, 1), b._Grid(32, 32, 1, 1, 1, 1), b._Grid(32, 32, 8, 1, 0, 1),
              b._Grid(32, 32, 600, 1, 1, 1), b._Grid(2, 32, 8, 1, 1, 1)):
        rc = lib.fvim_create(ctypes.byref(g), ctypes.byref(m), 0, 0, None, ctypes.byref(h))
        assert rc == b.FVIM_EINVAL
        assert lib.fvim_last_error()
    g = b._Grid(32, 32, 8, 1, 1, 1)
    bad = b._Material(1.0, 0.5, 0.01, 0.1)
    assert lib.fvim_create(ctypes.byref(g), ctypes.byref(bad), 0, 0, None, ctypes.byref(h)) == b.FVIM_EINVAL
    assert lib.fvim_create(ctypes.byref(g), ctypes.byref(m), 7, 0, None, ctypes.byref(h)) == b.FVIM_EINVAL
    assert lib.fvim_footprint_bytes(ctypes.byref(g), 0, 0) > 0
    assert lib.fvim_footprint_bytes(ctypes.byref(b._Grid(30, 32, 8, 1, 1, 1)), 0, 0) == 0


# ---------------------------------------------------------------- binding
C_SIZES = {"int": 4, "int32_t": 4, "double": 8, "char": 1, "uint64_t": 8, "size_t": 8}


def header_structs():
    """{name: [(c type, field, array length or None)]} of the header's typedef structs."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"typedef struct\s*\{(.*?)\}\s*(\w+);", src, flags=re.S):
        fields = []
        for decl in m.group(1).split(";"):
            decl = decl.strip()
            if not decl:
                continue
            t, rest = re.match(r"((?:const\s+)?[A-Za-z_]\w*(?:\s*\*)*)\s+(.*)$", decl, flags=re.S).groups()
            for part in rest.split(","):
                stars, name, _, n = re.match(r"(\**)\s*(\w+)\s*(\[(\w+)\])?", part.strip()).groups()
                fields.append((t + stars, name, n))
        out[m.group(2)] = fields
    return out


def header_constants():
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    vals = dict((k, int(v)) for k, v in re.findall(r"\b(FVIM_\w+)\s*=\s*(-?\d+)", src))
    vals.update((k, int(v)) for k, v in re.findall(r"#define\s+(FVIM_\w+)\s+(\d+)", src))
    return vals


def test_binding_structures_match_the_header():
    """Every ctypes structure of the binding has the header's fields, in the
    header's order and with the header's sizes, so the two layouts agree."""
    import ctypes as ct
    from paper_1811_11558_amd import binding as b
    pairs = {"fvim_grid": b._Grid, "fvim_material": b._Material, "fvim_contact_info": b._ContactInfo,
             "fvim_ep_opts": b.EPOptions, "fvim_ep_info": b._EPInfo, "fvim_request": b._Request,
             "fvim_result": b._Result, "fvim_server_stats": b._ServerStats,
             "fvim_tangential_info": b._TangentialInfo}
    consts = header_constants()
    hs = header_structs()
    for cname, py in pairs.items():
        fields = hs[cname]
        assert [f[1] for f in fields] == [f[0] for f in py._fields_], cname
        for (ctype, name, n), (_, pytype) in zip(fields, py._fields_):
            if ctype.endswith("*"):
                size = 8
            elif ctype in C_SIZES:
                size = C_SIZES[ctype]
            else:
                size = ct.sizeof(pairs[ctype])
            if n is not None:
                size *= consts[n] if n in consts else int(n)
            assert ct.sizeof(pytype) == size, (cname, name)


def test_binding_constants_match_the_header():
    """Option keys, status codes, precisions and the step limit of the
    binding are the header's values."""
    from paper_1811_11558_amd import binding as b
    c = header_constants()
    for name in ("DEPTH_CONFIG", "TUNE", "GRAPHS", "SIDE_STREAM", "STREAMING", "FFT_CONFIG"):
        assert getattr(b.Context, "OPT_" + name) == c["FVIM_OPT_" + name], name
    assert b.MAX_STEPS == c["FVIM_MAX_STEPS"]
    assert len(b.Context.STAGES) == c["FVIM_NSTAGES"]
    for name in ("OK", "EINVAL", "ENOMEM", "EHIP", "ENOCONV", "ENODEV"):
        assert getattr(b, "FVIM_" + name) == c["FVIM_" + name], name
    assert b.PRECISION == {"fp64": c["FVIM_FP64"], "fp32_refined": c["FVIM_FP32_REFINED"]}


def test_fft_config_packing_round_trips():
    """The binding's packing of the transform choices is the header's
    layout: 3 bits per kernel, tile | 4 for radix 8, default 0x249."""
    from paper_1811_11558_amd import binding as b
    assert b.pack_fft_config([(1, 4)] * 4) == 0x249
    cfg = [(0, 8), (2, 4), (1, 8), (0, 4)]
    assert b.unpack_fft_config(b.pack_fft_config(cfg)) == cfg
