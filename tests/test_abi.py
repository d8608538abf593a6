"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-only entry points (layout, workspace size,
table validation) behave as documented.  No compute call is made here."""
import ctypes as C
import os
import re

import pytest

from paper_1710_09995_amd import binding as B
from paper_1710_09995_amd import cases

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "cfd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cfd_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.EXPORTS)


def test_layout_alignment_and_disjoint_blocks():
    dims = [(17, 5, 3), (64, 2, 2), (3, 9, 4)]
    off, strides, total = B.layout(dims)
    end = 0
    for (ni, nj, nk), o, (sv, sk, sj, si) in zip(dims, off, strides):
        assert si == 1 and sj >= ni + 4 and sj % 16 == 0
        assert sk == sj * (nj + 4) and sv == sk * (nk + 4)
        assert (o + 2) % 16 == 0            # interior i = 0 on 128 bytes
        assert o >= end
        end = o + 5 * sv
    assert total >= end


def test_workspace_size_positive():
    c = cases.vortex_case(8)
    ws = C.c_size_t()
    st = B.lib().cfd_workspace_size(C.byref(B.to_params(c.params)), 1, B.to_dims(c.dims), C.byref(ws))
    assert st == 0 and ws.value > 10 * 8 * 12 ** 3


def _create(case, conns=None, bcs=None, params=None):
    """Call cfd_create_blocks with tables only; node/workspace pointers are
    placeholders that validation rejects before any device access."""
    L = B.lib()
    conns = case.conns if conns is None else conns
    bcs = case.bcs if bcs is None else bcs
    p = B.to_params(case.params if params is None else params)
    fake = (C.c_void_p * case.nblk)(*([0x1000] * case.nblk))
    ctx = C.c_void_p()
    st = L.cfd_create_blocks(C.byref(p), case.nblk, B.to_dims(case.dims), fake, len(conns), B.to_conns(conns),
                             len(bcs), B.to_bcs(bcs), None, C.c_size_t(0), None, C.byref(ctx))
    return st, L.cfd_last_error(None).decode()


def test_validation_rejects_double_cover():
    c = cases.vortex_case(4)
    extra = [cases.BC(0, 0, cases.FARFIELD, (0, 0), (1, 1))]
    st, msg = _create(c, bcs=extra)
    assert st == -1 and "covered twice" in msg


def test_validation_rejects_uncovered_face():
    c = cases.vortex_case(4)
    st, msg = _create(c, conns=c.conns[:-1])
    assert st == -1 and "not fully covered" in msg


def test_validation_rejects_same_side_connection():
    c = cases.vortex_case(4)
    conns = list(c.conns)
    a = conns[0]
    conns[0] = cases.Conn(a.blk, a.face, a.nbr, a.face, a.lo, a.hi, a.nbr_lo, a.shift)
    st, msg = _create(c, conns=conns)
    assert st == -1 and "opposite faces" in msg


def test_validation_rejects_out_of_range_patch_and_small_blocks():
    c = cases.vortex_case(4)
    bcs = [cases.BC(0, 0, cases.FARFIELD, (0, 0), (5, 4))]
    st, msg = _create(c, conns=[x for x in c.conns if x.face != 0], bcs=bcs)
    assert st == -1 and "outside face" in msg
    d = cases.vortex_case(4)
    d.dims[0] = (1, 4, 4)
    st, msg = _create(d)
    assert st == -1 and ">= 2" in msg


def test_unsupported_ghost_layers():
    c = cases.vortex_case(4)
    p = cases.Params(ghost_layers=3)
    st, msg = _create(c, params=p)
    assert st == -6


def test_status_strings():
    L = B.lib()
    for s in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.cfd_status_string(s)


def test_staggered_diff6_rejects_bad_arguments():
    """Argument checks of cfd_staggered_diff6 (each fails before any device
    access; the pointers are placeholders)."""
    L = B.lib()
    f, o = C.c_void_p(0x100000), C.c_void_p(0x900000)
    n = (C.c_int32 * 3)(8, 4, 2)
    ok = dict(f=f, o=o, n=n, d=0, nvar=5, h=0.1)
    bad = [dict(d=3), dict(d=-1), dict(nvar=0), dict(nvar=65), dict(h=0.0), dict(h=float("nan")),
           dict(n=(C.c_int32 * 3)(8, 0, 2)), dict(f=None), dict(o=C.c_void_p(0x100000 + 8 * 100))]
    for b in bad:
        a = dict(ok, **b)
        st = L.cfd_staggered_diff6(a["f"], a["o"], a["n"], a["d"], a["nvar"], a["h"], None)
        assert st == -1, b


def test_wcns5_edges_rejects_bad_arguments():
    """Argument checks of cfd_wcns5_edges (each fails before any device
    access; the pointers are placeholders)."""
    L = B.lib()
    u, lft, rgt = C.c_void_p(0x100000), C.c_void_p(0x900000), C.c_void_p(0x1100000)
    n = (C.c_int32 * 3)(8, 4, 2)
    ok = dict(u=u, l=lft, r=rgt, n=n, d=0, nvar=5, eps=1e-6)
    bad = [dict(d=3), dict(nvar=0), dict(eps=0.0), dict(eps=float("inf")), dict(n=(C.c_int32 * 3)(0, 4, 2)),
           dict(r=None), dict(r=lft), dict(l=C.c_void_p(0x100000 + 8 * 10))]
    for b in bad:
        a = dict(ok, **b)
        st = L.cfd_wcns5_edges(a["u"], a["l"], a["r"], a["n"], a["d"], a["nvar"], a["eps"], None)
        assert st == -1, b


def test_wcns5_residual_work_bytes_and_bad_arguments():
    L = B.lib()
    n = (C.c_int32 * 3)(8, 4, 2)
    nb = C.c_size_t()
    assert L.cfd_wcns5_euler_work_bytes(n, C.byref(nb)) == 0
    # the largest padded direction is k (2 cells: 32 lines of 2 + 10 padded cells, 2 + 5 faces):
    # 5 * 32 * 12 padded primitives + 5 * 32 * 7 face fluxes
    assert nb.value == 8 * (5 * 32 * 12 + 5 * 32 * 7)
    q, r, w = C.c_void_p(0x100000), C.c_void_p(0x900000), C.c_void_p(0x1100000)
    h = (C.c_double * 3)(0.1, 0.1, 0.1)
    ok = dict(q=q, r=r, w=w, wb=nb.value, n=n, h=h, g=1.4, ef=0.1, eps=1e-6)
    bad = {-2: [dict(wb=nb.value - 8)],
           -1: [dict(g=1.0), dict(ef=-0.1), dict(eps=0.0), dict(h=(C.c_double * 3)(0.1, 0.0, 0.1)),
                dict(n=(C.c_int32 * 3)(8, 0, 2)), dict(r=q), dict(w=None)]}
    for st_want, cases_ in bad.items():
        for b in cases_:
            a = dict(ok, **b)
            st = L.cfd_wcns5_euler_residual_periodic(a["q"], a["r"], a["w"], a["wb"], a["n"], a["h"], a["g"],
                                                     a["ef"], a["eps"], None)
            assert st == st_want, b


def test_header_is_plain_c(tmp_path):
    """include/cfd.h compiles as C99 (a C ABI: no C++ in the declarations)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("gcc or the ROCm headers are not available")
    src = tmp_path / "t.c"
    src.write_text('#include "cfd.h"\nint main(void) { cfd_ctx* c = 0; return (int)cfd_destroy(c); }\n')
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                        "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include", "-fsyntax-only", str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_wcns5_steps_bad_arguments():
    L = B.lib()
    n = (C.c_int32 * 3)(8, 4, 2)
    nb, nr = C.c_size_t(), C.c_size_t()
    assert L.cfd_wcns5_euler_step_work_bytes(n, C.byref(nb)) == 0
    assert L.cfd_wcns5_euler_work_bytes(n, C.byref(nr)) == 0
    assert nb.value == nr.value + 2 * 40 * 64          # + start state and R: 5 doubles per cell each
    q, w = C.c_void_p(0x100000), C.c_void_p(0x900000)
    h = (C.c_double * 3)(0.1, 0.1, 0.1)
    for st_want, kw in ((-1, dict(dt=0.0)), (-1, dict(ns=-1)), (-2, dict(wb=nb.value - 8)), (-1, dict(w=None))):
        a = dict(q=q, w=w, wb=nb.value, dt=0.01, ns=1)
        a.update(kw)
        st = L.cfd_wcns5_euler_steps_periodic(a["q"], a["w"], a["wb"], n, h, 1.4, 0.1, 1e-6, a["dt"], a["ns"], None)
        assert st == st_want, kw


def test_c4_viscous_bad_arguments():
    L = B.lib()
    n = (C.c_int32 * 3)(8, 4, 2)
    nb = C.c_size_t()
    assert L.cfd_c4_viscous_work_bytes(n, C.byref(nb)) == 0 and nb.value == 8 * 20 * 64
    q, r, w = C.c_void_p(0x100000), C.c_void_p(0x900000), C.c_void_p(0x1100000)
    h = (C.c_double * 3)(0.1, 0.1, 0.1)
    for st_want, kw in ((-2, dict(wb=nb.value - 8)), (-1, dict(pr=0.0)), (-1, dict(mu=-1.0)), (-1, dict(r=q)),
                        (-1, dict(g=1.0))):
        a = dict(q=q, r=r, w=w, wb=nb.value, g=1.4, pr=0.72, mu=1e-3)
        a.update(kw)
        st = L.cfd_c4_viscous_add_periodic(a["q"], a["r"], a["w"], a["wb"], n, h, a["g"], a["pr"], a["mu"], 0.38,
                                           None)
        assert st == st_want, kw


def test_curvilinear_metrics_and_residual_bad_arguments():
    L = B.lib()
    n = (C.c_int32 * 3)(8, 4, 2)
    per = (C.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    xv, s, j = C.c_void_p(0x100000), C.c_void_p(0x900000), C.c_void_p(0x1100000)
    ok = dict(xv=xv, per=per, n=n, s=s, j=j)
    bad = [dict(xv=None), dict(per=None), dict(s=None), dict(j=None), dict(n=(C.c_int32 * 3)(8, 0, 2)),
           dict(per=(C.c_double * 9)(1, 0, 0, 0, float("nan"), 0, 0, 0, 1)), dict(s=xv),
           dict(j=C.c_void_p(0x900000 + 8 * 64))]
    for b in bad:
        a = dict(ok, **b)
        assert L.cfd_wcns5_metrics_periodic(a["xv"], a["per"], a["n"], a["s"], a["j"], None) == -1, b
    nb = C.c_size_t()
    assert L.cfd_wcns5_euler_work_bytes(n, C.byref(nb)) == 0
    q, r, w = C.c_void_p(0x2100000), C.c_void_p(0x2900000), C.c_void_p(0x3100000)
    ok = dict(q=q, s=s, j=j, r=r, w=w, wb=nb.value, n=n, g=1.4, ef=0.1, eps=1e-6)
    bad = {-2: [dict(wb=nb.value - 8)],
           -1: [dict(q=None), dict(s=None), dict(j=None), dict(r=None), dict(w=None), dict(g=1.0), dict(ef=-0.1),
                dict(eps=0.0), dict(n=(C.c_int32 * 3)(0, 4, 2)), dict(r=q), dict(r=s),
                dict(j=C.c_void_p(0x2900000 + 8 * 10)), dict(w=C.c_void_p(0x900000 + 8 * 100))]}
    for st_want, cases_ in bad.items():
        for b in cases_:
            a = dict(ok, **b)
            st = L.cfd_wcns5_euler_residual_curv_periodic(a["q"], a["s"], a["j"], a["r"], a["w"], a["wb"], a["n"],
                                                          a["g"], a["ef"], a["eps"], None)
            assert st == st_want, b


def test_curvilinear_steps_bad_arguments():
    L = B.lib()
    n = (C.c_int32 * 3)(8, 4, 2)
    nb = C.c_size_t()
    assert L.cfd_wcns5_euler_step_work_bytes(n, C.byref(nb)) == 0
    q, s, j, w = C.c_void_p(0x100000), C.c_void_p(0x900000), C.c_void_p(0x1100000), C.c_void_p(0x2100000)
    ok = dict(q=q, s=s, j=j, w=w, wb=nb.value, n=n, g=1.4, ef=0.1, eps=1e-6, dt=0.01, ns=2)
    bad = {-2: [dict(wb=nb.value - 8)],
           -1: [dict(q=None), dict(s=None), dict(j=None), dict(w=None), dict(dt=0.0), dict(ns=-1), dict(g=1.0),
                dict(n=(C.c_int32 * 3)(8, 4, 0)), dict(s=C.c_void_p(0x100000 + 8 * 4)),
                dict(w=C.c_void_p(0x100000 + 8))]}
    for st_want, cases_ in bad.items():
        for b in cases_:
            a = dict(ok, **b)
            st = L.cfd_wcns5_euler_steps_curv_periodic(a["q"], a["s"], a["j"], a["w"], a["wb"], a["n"], a["g"],
                                                       a["ef"], a["eps"], a["dt"], a["ns"], None)
            assert st == st_want, b


def test_curvilinear_viscous_bad_arguments():
    L = B.lib()
    n = (C.c_int32 * 3)(8, 4, 2)
    nb = C.c_size_t()
    assert L.cfd_c4_viscous_curv_work_bytes(n, C.byref(nb)) == 0
    assert nb.value == 8 * (16 + 21) * 64     # phi and gradients, face metrics
    q, s, j, r, w = (C.c_void_p(a) for a in (0x100000, 0x900000, 0x1100000, 0x2100000, 0x3100000))
    ok = dict(q=q, s=s, j=j, r=r, w=w, wb=nb.value, n=n, g=1.4, pr=0.72, mu=1e-3, ss=0.38)
    bad = {-2: [dict(wb=nb.value - 8)],
           -1: [dict(q=None), dict(s=None), dict(j=None), dict(r=None), dict(w=None), dict(g=1.0), dict(pr=0.0),
                dict(mu=-1.0), dict(ss=0.0), dict(n=(C.c_int32 * 3)(8, 4, 0)), dict(r=q), dict(r=s),
                dict(r=C.c_void_p(0x1100000 - 8)), dict(w=C.c_void_p(0x2100000 + 8))]}
    for st_want, cases_ in bad.items():
        for b in cases_:
            a = dict(ok, **b)
            st = L.cfd_c4_viscous_add_curv_periodic(a["q"], a["s"], a["j"], a["r"], a["w"], a["wb"], a["n"], a["g"],
                                                    a["pr"], a["mu"], a["ss"], None)
            assert st == st_want, b


def test_curvilinear_time_step_bad_arguments():
    L = B.lib()
    n = (C.c_int32 * 3)(8, 4, 2)
    q, s, j, dt = (C.c_void_p(a) for a in (0x100000, 0x900000, 0x1100000, 0x2100000))
    ok = dict(q=q, s=s, j=j, n=n, g=1.4, cfl=0.5, v=1, pr=0.72, mu=1e-3, ss=0.38, dt=dt)
    bad = [dict(q=None), dict(s=None), dict(j=None), dict(dt=None), dict(n=(C.c_int32 * 3)(0, 4, 2)), dict(g=1.0),
           dict(cfl=0.0), dict(cfl=float("inf")), dict(pr=0.0), dict(mu=-1.0), dict(ss=0.0),
           dict(dt=C.c_void_p(0x100000 + 8)), dict(dt=C.c_void_p(0x2100004))]
    for b in bad:
        a = dict(ok, **b)
        st = L.cfd_wcns5_time_step_curv_periodic(a["q"], a["s"], a["j"], a["n"], a["g"], a["cfl"], a["v"], a["pr"],
                                                 a["mu"], a["ss"], a["dt"], None)
        assert st == -1, b


def test_block_seams_bad_arguments():
    L = B.lib()
    # two blocks 8 x 6 x 5 side by side along i, each its own neighbour along j and k
    dims = (C.c_int32 * 6)(8, 6, 5, 8, 6, 5)
    nbr = (C.c_int32 * 12)(1, 1, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1)
    nb = C.c_size_t()
    assert L.cfd_wcns5_euler_blocks_work_bytes(2, dims, nbr, C.byref(nb)) == 0
    # largest padded direction k (5 + 10 cells, 5 + 5 faces over 48 lines): 5*48*15 + 5*48*10
    assert nb.value == 8 * (5 * 48 * 15 + 5 * 48 * 10)
    bad_tables = [(C.c_int32 * 12)(1, 1, 0, 0, 0, 0, 0, 0, 1, 1, 1, 2),      # out of range
                  (C.c_int32 * 12)(1, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1)]      # not mutual
    for t in bad_tables:
        assert L.cfd_wcns5_euler_blocks_work_bytes(2, dims, t, C.byref(nb)) == -1
    assert L.cfd_wcns5_euler_blocks_work_bytes(2, (C.c_int32 * 6)(8, 6, 5, 8, 7, 5), nbr, C.byref(nb)) == -1
    assert L.cfd_wcns5_euler_blocks_work_bytes(2, (C.c_int32 * 6)(8, 6, 4, 8, 6, 4), nbr, C.byref(nb)) == -1
    assert L.cfd_wcns5_euler_blocks_work_bytes(0, dims, nbr, C.byref(nb)) == -1
    assert L.cfd_wcns5_euler_blocks_work_bytes(2, dims, nbr, C.byref(nb)) == 0
    P = lambda *a: (C.c_void_p * 2)(*[C.c_void_p(v) for v in a])         # noqa: E731
    q, s, j, r = P(0x100000, 0x200000), P(0x300000, 0x400000), P(0x500000, 0x600000), P(0x700000, 0x800000)
    w = C.c_void_p(0x900000)
    ok = dict(q=q, s=s, j=j, r=r, w=w, wb=nb.value, g=1.4, ef=0.1, eps=1e-6)
    bad = {-2: [dict(wb=nb.value - 8)],
           -1: [dict(q=None), dict(w=None), dict(g=1.0), dict(eps=0.0), dict(r=P(0x700000, 0x700000 + 8)),
                dict(r=P(0x100000, 0x800000)), dict(w=C.c_void_p(0x500000)), dict(q=P(0x100000, 0))]}
    for st_want, cases_ in bad.items():
        for b in cases_:
            a = dict(ok, **b)
            st = L.cfd_wcns5_euler_residual_blocks(2, dims, nbr, a["q"], a["s"], a["j"], a["r"], a["w"], a["wb"],
                                                   a["g"], a["ef"], a["eps"], None)
            assert st == st_want, b
    xe = C.c_void_p(0x100000)
    n = (C.c_int32 * 3)(8, 6, 5)
    for b in (dict(xe=None), dict(s=None), dict(n=(C.c_int32 * 3)(8, 0, 6)), dict(s=xe)):
        a = dict(dict(xe=xe, n=n, s=C.c_void_p(0x900000), j=C.c_void_p(0xA00000)), **b)
        assert L.cfd_wcns5_metrics_ext(a["xe"], a["n"], a["s"], a["j"], None) == -1, b


def test_viscous_seams_bad_arguments():
    L = B.lib()
    dims = (C.c_int32 * 6)(8, 6, 5, 8, 6, 5)
    nbr = (C.c_int32 * 12)(1, 1, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1)
    nb = C.c_size_t()
    assert L.cfd_c4_viscous_blocks_work_bytes(2, dims, nbr, C.byref(nb)) == 0
    assert nb.value == 8 * (16 + 21) * 240 * 2
    bad_nbr = (C.c_int32 * 12)(1, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1)
    assert L.cfd_c4_viscous_blocks_work_bytes(2, dims, bad_nbr, C.byref(nb)) == -1
    assert L.cfd_c4_viscous_blocks_work_bytes(2, dims, nbr, C.byref(nb)) == 0
    P = lambda *a: (C.c_void_p * 2)(*[C.c_void_p(v) for v in a])         # noqa: E731
    q, s, j, r = P(0x100000, 0x200000), P(0x300000, 0x400000), P(0x500000, 0x600000), P(0x700000, 0x800000)
    w = C.c_void_p(0x900000)
    ok = dict(q=q, s=s, j=j, r=r, w=w, wb=nb.value, g=1.4, pr=0.72, mu=1e-3, ss=0.38)
    bad = {-2: [dict(wb=nb.value - 8)],
           -1: [dict(q=None), dict(w=None), dict(g=1.0), dict(pr=0.0), dict(mu=-1.0),
                dict(r=P(0x700000, 0x700000 + 8)), dict(r=P(0x300000, 0x800000)), dict(w=C.c_void_p(0x600000)),
                dict(j=P(0x500000, 0))]}
    for st_want, cases_ in bad.items():
        for b in cases_:
            a = dict(ok, **b)
            st = L.cfd_c4_viscous_add_blocks(2, dims, nbr, a["q"], a["s"], a["j"], a["r"], a["w"], a["wb"], a["g"],
                                             a["pr"], a["mu"], a["ss"], None)
            assert st == st_want, b


def test_ns_steps_bad_arguments():
    L = B.lib()
    n = (C.c_int32 * 3)(8, 4, 2)
    nb = C.c_size_t()
    assert L.cfd_wcns5_ns_step_work_bytes(n, C.byref(nb)) == 0
    # the larger scratch (16 doubles per cell for the viscous terms vs the residual's), the viscous face
    # metrics (21 per cell), start state and R
    assert nb.value == max(8 * (5 * 32 * 12 + 5 * 32 * 7), 8 * 16 * 64) + 8 * 21 * 64 + 2 * 40 * 64
    q, s, j, w = C.c_void_p(0x100000), C.c_void_p(0x900000), C.c_void_p(0x1100000), C.c_void_p(0x2100000)
    ok = dict(q=q, s=s, j=j, w=w, wb=nb.value, g=1.4, ef=0.1, eps=1e-6, pr=0.72, mu=1e-3, ss=0.38, dt=0.01, ns=2)
    bad = {-2: [dict(wb=nb.value - 8)],
           -1: [dict(q=None), dict(s=None), dict(w=None), dict(g=1.0), dict(pr=0.0), dict(mu=-1.0), dict(ss=0.0),
                dict(dt=0.0), dict(ns=-1), dict(w=C.c_void_p(0x100000 + 8))]}
    for st_want, cases_ in bad.items():
        for b in cases_:
            a = dict(ok, **b)
            st = L.cfd_wcns5_ns_steps_curv_periodic(a["q"], a["s"], a["j"], a["w"], a["wb"], n, a["g"], a["ef"],
                                                    a["eps"], a["pr"], a["mu"], a["ss"], a["dt"], a["ns"], None)
            assert st == st_want, b


def test_implicit_steps_bad_arguments():
    L = B.lib()
    n = (C.c_int32 * 3)(8, 4, 2)
    nb = C.c_size_t()
    assert L.cfd_wcns5_implicit_step_work_bytes(n, C.byref(nb)) == 0
    # the larger scratch (the viscous terms' 16 doubles per cell, or the residual's) + the face metrics
    # (21) + 22 doubles per cell
    assert nb.value == max(8 * (5 * 32 * 12 + 5 * 32 * 7), 8 * 16 * 64) + 8 * 21 * 64 + 8 * 22 * 64
    q, s, j, w = C.c_void_p(0x100000), C.c_void_p(0x900000), C.c_void_p(0x1100000), C.c_void_p(0x2100000)
    ok = dict(q=q, s=s, j=j, w=w, wb=nb.value, g=1.4, ef=0.1, eps=1e-6, v=1, pr=0.72, mu=1e-3, ss=0.38, dt=0.01,
              ns=2, sw=3)
    bad = {-2: [dict(wb=nb.value - 8)],
           -1: [dict(q=None), dict(s=None), dict(j=None), dict(w=None), dict(g=1.0), dict(dt=0.0), dict(ns=-1),
                dict(sw=-1), dict(sw=1001), dict(w=C.c_void_p(0x100000 + 8)), dict(s=C.c_void_p(0x100000 + 8)),
                dict(w=C.c_void_p(0x1100000 - 8)), dict(pr=0.0), dict(mu=-1.0), dict(ss=0.0)]}
    for st_want, cases_ in bad.items():
        for b in cases_:
            a = dict(ok, **b)
            st = L.cfd_wcns5_implicit_steps_curv_periodic(a["q"], a["s"], a["j"], a["w"], a["wb"], n, a["g"], a["ef"],
                                                          a["eps"], a["v"], a["pr"], a["mu"], a["ss"], a["dt"],
                                                          a["ns"], a["sw"], None)
            assert st == st_want, b


def test_implicit_blocks_bad_arguments():
    L = B.lib()
    dims = (C.c_int32 * 6)(8, 6, 5, 8, 6, 5)
    nbr = (C.c_int32 * 12)(1, 1, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1)
    nb = C.c_size_t()
    assert L.cfd_wcns5_implicit_blocks_work_bytes(2, dims, nbr, C.byref(nb)) == 0
    assert nb.value == max(8 * (5 * 48 * 15 + 5 * 48 * 10), 8 * 16 * 480) + 8 * (21 + 22) * 480
    P = lambda *a: (C.c_void_p * 2)(*[C.c_void_p(v) for v in a])         # noqa: E731
    q, s, j = P(0x100000, 0x200000), P(0x300000, 0x400000), P(0x500000, 0x600000)
    w = C.c_void_p(0x900000)
    ok = dict(q=q, s=s, j=j, w=w, wb=nb.value, g=1.4, ef=0.1, eps=1e-6, v=1, pr=0.72, mu=1e-3, ss=0.38, dt=0.01,
              ns=1, sw=2)
    bad = {-2: [dict(wb=nb.value - 8)],
           -1: [dict(q=None), dict(w=None), dict(g=1.0), dict(dt=0.0), dict(sw=-1), dict(ns=-1), dict(pr=0.0),
                dict(q=P(0x100000, 0x100000 + 8)), dict(q=P(0x300000, 0x200000)), dict(w=C.c_void_p(0x500000)),
                dict(j=P(0x500000, 0))]}
    for st_want, cases_ in bad.items():
        for b in cases_:
            a = dict(ok, **b)
            st = L.cfd_wcns5_implicit_steps_blocks(2, dims, nbr, a["q"], a["s"], a["j"], a["w"], a["wb"], a["g"],
                                                   a["ef"], a["eps"], a["v"], a["pr"], a["mu"], a["ss"], a["dt"],
                                                   a["ns"], a["sw"], None)
            assert st == st_want, b


def test_ns_blocks_bad_arguments():
    L = B.lib()
    dims = (C.c_int32 * 6)(8, 6, 5, 8, 6, 5)
    nbr = (C.c_int32 * 12)(1, 1, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1)
    nb = C.c_size_t()
    assert L.cfd_wcns5_ns_blocks_work_bytes(2, dims, nbr, C.byref(nb)) == 0
    assert nb.value == max(8 * (5 * 48 * 15 + 5 * 48 * 10), 8 * 16 * 480) + 8 * (10 + 21) * 480
    P = lambda *a: (C.c_void_p * 2)(*[C.c_void_p(v) for v in a])         # noqa: E731
    q, s, j = P(0x100000, 0x200000), P(0x300000, 0x400000), P(0x500000, 0x600000)
    w = C.c_void_p(0x900000)
    ok = dict(q=q, s=s, j=j, w=w, wb=nb.value, g=1.4, ef=0.1, eps=1e-6, pr=0.72, mu=1e-3, ss=0.38, dt=0.01, ns=1)
    bad = {-2: [dict(wb=nb.value - 8)],
           -1: [dict(q=None), dict(w=None), dict(g=1.0), dict(pr=0.0), dict(mu=-1.0), dict(dt=0.0), dict(ns=-1),
                dict(q=P(0x100000, 0x100000 + 8)), dict(w=C.c_void_p(0x500000))]}
    for st_want, cases_ in bad.items():
        for b in cases_:
            a = dict(ok, **b)
            st = L.cfd_wcns5_ns_steps_blocks(2, dims, nbr, a["q"], a["s"], a["j"], a["w"], a["wb"], a["g"], a["ef"],
                                             a["eps"], a["pr"], a["mu"], a["ss"], a["dt"], a["ns"], None)
            assert st == st_want, b


def _self_joined(nblk, n=5):
    """nblk blocks of n^3 cells, each its own neighbour across every face."""
    dims = (C.c_int32 * (3 * nblk))(*([n, n, n] * nblk))
    nbr = (C.c_int32 * (6 * nblk))(*[b for b in range(nblk) for _ in range(6)])
    return dims, nbr


def _fake_spans(nblk, sizes, base=1 << 40):
    """Disjoint fake device addresses (never dereferenced: every call below
    fails its argument checks before any launch), 256-byte aligned."""
    out, at = [], base
    for size in sizes:
        ptrs = []
        for _ in range(nblk):
            ptrs.append(at)
            at += (size + 255) // 256 * 256
        out.append(ptrs)
    return out, at


@pytest.mark.parametrize("nblk", [3, 65536])
def test_block_entry_points_reject_overlapping_buffers(nblk):
    """The joined-block entry points check every pair of buffers for overlap
    (in O(n log n): 65536 blocks take well under a second) and refuse a
    written buffer that overlaps any other before launching anything."""
    import time
    L = B.lib()
    vp = C.c_void_p
    dims, nbr = _self_joined(nblk)
    cells = 125
    need = C.c_size_t()
    B._check(L.cfd_wcns5_euler_blocks_work_bytes(nblk, dims, nbr, C.byref(need)))
    (q, s, j, r), end = _fake_spans(nblk, [40 * cells, 72 * cells, 8 * cells, 40 * cells])
    arr = lambda v: (vp * nblk)(*v)   # noqa: E731

    def residual(q, s, j, r, work):
        return L.cfd_wcns5_euler_residual_blocks(nblk, dims, nbr, arr(q), arr(s), arr(j), arr(r), work,
                                                 need.value, 1.4, 0.1, 1e-6, None)
    cases_ = [
        (q, s, j, r[:-1] + [q[0] + 8], end),             # last residual inside the first state
        (q, s, j, r[:-1] + [r[0] + 40 * cells - 8], end),  # two residuals share 8 bytes
        (q, s, j, r, s[nblk // 2]),                        # the workspace starts inside a face-metric array
    ]
    for args in cases_:
        t0 = time.perf_counter()
        st = residual(*args)
        assert st == -1 and "overlaps" in L.cfd_last_error(None).decode(), st
        assert time.perf_counter() - t0 < 5.0
    iw = C.c_size_t()
    B._check(L.cfd_wcns5_implicit_blocks_work_bytes(nblk, dims, nbr, C.byref(iw)))
    st = L.cfd_wcns5_implicit_steps_blocks(nblk, dims, nbr, arr(q[:-1] + [q[0] + 16]), arr(s), arr(j), end,
                                           iw.value, 1.4, 0.1, 1e-6, 0, 0.72, 0.0, 0.38, 1e-3, 1, 2, None)
    assert st == -1 and "overlaps" in L.cfd_last_error(None).decode()
