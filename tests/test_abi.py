"""C-ABI contract of libsnowlb, CPU only: the library loads, exports every function the header
declares, and rejects invalid parameters before any GPU call."""
import ctypes
import os
import re

import pytest

from paper_2101_07163_amd import snowlb as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    """Every function declared in include/*.h (comments stripped)."""
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(snowlb(?:3d)?_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_header_symbols_exported_and_bound():
    L = S.lib()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n           # exported by the shared library
        assert n in S._SIGS, n            # bound by the Python binding with the same name


def test_status_strings():
    for code, name in ((0, "SNOWLB_OK"), (-1, "SNOWLB_EINVAL"), (-5, "SNOWLB_ENONFINITE"),
                       (-6, "SNOWLB_ESTATE")):
        assert S.lib().snowlb_status_str(code).decode() == name


def test_defaults_are_valid():
    p = S.snowlb_params_default()
    assert S.snowlb_validate(p) == (0, "")
    assert (p.nx, p.ny, p.n_fold) == (128, 128, 6)
    assert (p.stencil, p.symmetric) == (4, 0)


@pytest.mark.parametrize("field,value,frag", [
    ("nx", 1, "nx and ny"), ("ny", 0, "nx and ny"), ("tau_vap", 0.5, "tau_vap"),
    ("n_fold", 5, "n_fold"), ("storage", 3, "storage"), ("eps", 0.6, "eps"),
    ("W0", 0.0, "W0"), ("tile", 99, "tile"), ("diag_every", -1, "diag_every"),
    ("eps", float("nan"), "non-finite"), ("init_width", 0.0, "init_width"),
    ("stencil", 3, "stencil"), ("stencil", 0, "stencil"), ("symmetric", 2, "symmetric"),
])
def test_invalid_params_rejected_before_gpu(field, value, frag):
    p = S.snowlb_params_default()
    setattr(p, field, value)
    st, msg = S.snowlb_validate(p)
    assert st == S.EINVAL and frag in msg
    ctx = ctypes.c_void_p(123)
    st = S.lib().snowlb_create(ctypes.byref(p), ctypes.byref(ctx))
    assert st == S.EINVAL and not ctx.value
    assert frag in S.lib().snowlb_last_error(None).decode()


def test_flow_dependent_rules():
    p = S.snowlb_params_default()
    p.bc_x = S.BC_INOUT
    assert S.snowlb_validate(p)[0] == S.EINVAL       # inflow/outflow needs the flow solver
    p.flow = 1
    assert S.snowlb_validate(p)[0] == S.OK
    p.u_in = 0.2
    assert S.snowlb_validate(p)[0] == S.EINVAL       # Mach limit
    p.u_in = 0.01
    p.tau_f = 0.5
    assert S.snowlb_validate(p)[0] == S.EINVAL


def test_null_arguments():
    L = S.lib()
    assert L.snowlb_create(None, None) == S.EINVAL
    assert L.snowlb_step(None, 1, None) == S.EINVAL
    assert L.snowlb_step_count(None) == -1
    L.snowlb_destroy(None)


def test_tile_configurations():
    n = S.snowlb_tile_count()
    assert n >= 4
    names = [S.snowlb_tile_name(i) for i in range(n)]
    assert all(re.fullmatch(r"\d+x\d+", s) for s in names)
    assert S.lib().snowlb_tile_name(n).decode() == "?"


def test_batch_rejects_mixed_kernels_before_gpu():
    a = S.snowlb_params_default()
    b = S.snowlb_params_default()
    b.flow = 1
    arr = (S.snowlb_params * 2)(a, b)
    out = ctypes.c_void_p(7)
    assert S.lib().snowlb_batch_create(arr, 2, ctypes.byref(out)) == S.EINVAL and not out.value
    assert "share" in S.lib().snowlb_batch_last_error(None).decode()
    a.nx = 1
    arr = (S.snowlb_params * 2)(a, a)
    assert S.lib().snowlb_batch_create(arr, 2, ctypes.byref(out)) == S.EINVAL
    assert "domain 0" in S.lib().snowlb_batch_last_error(None).decode()
    assert S.lib().snowlb_batch_create(arr, 0, ctypes.byref(out)) == S.EINVAL
    # E2 and E4 share a kernel (one-cell halo); E4 and E8 do not
    a = S.snowlb_params_default()
    b = S.snowlb_params_default()
    b.stencil = 8
    arr = (S.snowlb_params * 2)(a, b)
    assert S.lib().snowlb_batch_create(arr, 2, ctypes.byref(out)) == S.EINVAL and not out.value
    assert "stencil" in S.lib().snowlb_batch_last_error(None).decode()


def test_lattice_size_limit():
    """Every byte offset of the step kernel inside one buffer is 32-bit: the populations of one copy
    (with the 16-bit reference planes in 16-bit storage), on the lattice padded to whole 64 x 4
    blocks, must fit in 4 GiB: 23 planes with flow and 14 without at 4 B in FP32; 27 and 15 planes at
    2 B in 16-bit storage.  Checked on the host, before any GPU call."""
    def padded(n, m):
        return -(-n // m) * m

    for flow in (0, 1):
        for storage, esize in ((S.STORE_FP32, 4), (S.STORE_FP16, 2)):
            per_cell = (23 if flow else 14) * 4 if esize == 4 else (27 if flow else 15) * 2
            # the widest square lattice that fits, and one block row more
            n = 64
            while padded(n + 64, 64) * padded(n + 64, 4) * per_cell <= 1 << 32:
                n += 64
            p = S.snowlb_params_default()
            p.flow, p.storage = flow, storage
            p.nx, p.ny = n, n
            assert S.snowlb_validate(p) == (0, ""), (flow, storage, n)
            ny = n
            while padded(n, 64) * padded(ny, 4) * per_cell <= 1 << 32:
                ny += 4
            p.ny = ny
            st, msg = S.snowlb_validate(p)
            assert st == S.EINVAL and "too large" in msg, (flow, storage, n, ny)
    p = S.snowlb_params_default()
    p.nx, p.ny = 65537, 8
    assert S.snowlb_validate(p)[0] == S.EINVAL


def test_diagnostics_count_matches_header():
    """snowlb_diag fills SNOWLB_DIAG_COUNT doubles (the eight sums and the species invariant); the
    binding's buffer has exactly that many."""
    txt = open(os.path.join(ROOT, "include", "snowlb.h")).read()
    m = re.search(r"#define\s+SNOWLB_DIAG_COUNT\s+(\d+)", txt)
    assert m and int(m.group(1)) == S.DIAG_COUNT == len(S.DIAG_KEYS) == 9
    assert S.DIAG_KEYS[8] == "species"


def test_3d_parameters_validated_before_gpu():
    """The 3D entry points validate like the 2D ones: defaults are valid, and out-of-range values are
    rejected with a message before any GPU call (snowlb3d_create fails with EINVAL and a NULL ctx)."""
    assert "snowlb3d_step" in header_functions() and "snowlb3d_diag" in header_functions()
    p = S.snowlb3d_params_default()
    assert S.snowlb3d_validate(p) == (0, "")
    assert (p.nx, p.ny, p.nz, p.flow) == (64, 64, 64, 0)
    for field, value, frag in (("nz", 1, "nz"), ("tau_vap", 0.5, "tau_vap"), ("eps", 0.5, "eps"),
                               ("bc_x", 1, "inflow/outflow"), ("init_width", 0.0, "init_width"),
                               ("nx", 4096, "too large")):
        q = S.snowlb3d_params_default()
        setattr(q, field, value)
        if field == "nx":
            q.ny, q.nz, q.flow = 4096, 64, 1
        st, msg = S.snowlb3d_validate(q)
        assert st == S.EINVAL and frag in msg, (field, msg)
        ctx = ctypes.c_void_p(123)
        assert S.lib().snowlb3d_create(ctypes.byref(q), ctypes.byref(ctx)) == S.EINVAL and not ctx.value
        assert frag in S.lib().snowlb3d_last_error(None).decode()
    assert S.lib().snowlb3d_step(None, 1, None) == S.EINVAL and S.lib().snowlb3d_step_count(None) == -1
