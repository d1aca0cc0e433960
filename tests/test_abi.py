"""The C-ABI library loads on a host without a GPU, exports every entry point
declared in include/grmhd.h, and validates its arguments host-side (no
compute call is made here)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "grmhd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(grmhd_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1102_5202_amd import grmhd
    if not os.path.exists(grmhd.LIB_PATH):
        from paper_1102_5202_amd import build
        build.build()
    return grmhd


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) == 31, names
    assert set(names) == set(lib.SYMBOLS)
    L = lib.load()
    for n in names:
        assert hasattr(L, n)
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (grmhd_\w+)", out))
    assert set(names) <= exported


def _host_ws(nbytes):
    raw = np.zeros(nbytes + 512, dtype=np.uint8)
    addr = raw.ctypes.data
    off = (-addr) % 256
    return raw, addr + off


def test_workspace_and_init_validation(lib):
    L = lib.load()
    g = lib.make_grid((16, 8, 1), (0, 0, 0), (1, 1, 1), (0, 1, 1))
    nb = L.grmhd_workspace_bytes(C.byref(g), None)
    # counters + ghosted cache + stage buffer + x and y face fluxes
    px = ((16 + 4 + 7) // 8) * 8
    assert nb >= 8 * 9 * (px * 12 * 1 + 16 * 8 + 17 * 8 + 16 * 9)
    bad = lib.make_grid((0, 8, 1), (0, 0, 0), (1, 1, 1), (0, 0, 0))
    assert L.grmhd_workspace_bytes(C.byref(bad), None) == 0
    # sizes whose byte counts would overflow are refused, not wrapped
    huge = lib.make_grid((1 << 20, 1 << 20, 1 << 20), (0, 0, 0), (1, 1, 1), (0, 0, 0))
    assert L.grmhd_workspace_bytes(C.byref(huge), None) == 0
    big = lib.make_grid((1 << 19, 1 << 19, 1), (0, 0, 0), (1, 1, 1), (0, 0, 0))
    assert L.grmhd_workspace_bytes(C.byref(big), None) > 9 * 8 * (1 << 38)
    raw, addr = _host_ws(nb)
    m = lib.Metric(lib.FLAT, 0, 0.0, 1.0)
    e = lib.Eos(0, 5.0 / 3.0, 0.0)

    def init(opts, metric=m, eos=e, grid=g):
        ctx = C.c_void_p()
        rc = L.grmhd_init(C.byref(ctx), C.byref(metric), C.byref(grid), C.byref(eos), C.byref(opts))
        if rc == 0:
            assert L.grmhd_free(ctx) == 0
        return rc

    ok = lib.Opts(3, 0, 1.0, 1.0, 1e-12, 1e-12, 1e-12, 50, 0, 0, 0, 0, 0, 0, C.c_void_p(addr), nb)
    assert init(ok) == 0
    assert init(lib.Opts(4, 0, 1.0, 1.0, 1e-12, 1e-12, 1e-12, 50, 0, 0, 0, 0, 0, 0, C.c_void_p(addr), nb)) == -1
    assert init(lib.Opts(3, 0, 1.0, 1.0, 1e-12, 1e-12, 1e-12, 50, 0, 0, 0, 0, 0, 0, C.c_void_p(addr), nb - 8)) == -2
    assert init(lib.Opts(3, 0, 1.0, 1.0, 1e-12, 1e-12, 1e-12, 50, 0, 0, 0, 0, 0, 0, C.c_void_p(addr + 8), nb)) == -2
    assert init(lib.Opts(3, 0, 1.0, 1.0, 1e-12, 1e-12, 1e-12, 50, 0, 0, 0, 0, 0, 0, None, nb)) == -2
    assert init(lib.Opts(3, 0, 1.0, 1.0, 0.0, 1e-12, 1e-12, 50, 0, 0, 0, 0, 0, 0, C.c_void_p(addr), nb)) == -1
    assert init(lib.Opts(3, 0, 1.0, 1.0, 1e-12, 1e-12, 1e-12, 50, 2, 0, 0, 0, 0, 0, C.c_void_p(addr), nb)) == -1
    assert init(lib.Opts(3, 0, 1.0, 1.0, 1e-12, 1e-12, 1e-12, 50, 1, 0, 0, 0, 0, 0, C.c_void_p(addr), nb)) == 0
    assert init(ok, eos=lib.Eos(0, 2.5, 0.0)) == -1
    assert init(ok, metric=lib.Metric(lib.ISO_SCHW, 0, 1.0, 0.4)) == -1   # r_min <= M/2
    assert init(ok, metric=lib.Metric(lib.ISO_SCHW, 0, 1.0, 1.0)) == 0
    assert init(ok, metric=lib.Metric(7, 0, 1.0, 1.0)) == -1
    for code in (0, -1, -2, -3, -4, -5, -99):
        assert L.grmhd_strerror(code)
    # calls out of order are refused before any device work
    ctx = C.c_void_p()
    assert L.grmhd_init(C.byref(ctx), C.byref(m), C.byref(g), C.byref(e), C.byref(ok)) == 0
    assert L.grmhd_step(ctx, C.c_void_p(addr), C.c_double(0.1)) == -4
    assert L.grmhd_step(ctx, None, C.c_double(0.1)) == -1
    assert L.grmhd_cons(ctx, None, None) == -1
    # adjoint calls on a context without the adjoint workspace
    p = C.c_void_p(addr)
    assert L.grmhd_step_adjoint(ctx, p, p, C.c_double(0.1)) == -5
    assert L.grmhd_prim_adjoint(ctx, p, p, p) == -5
    assert L.grmhd_cons_adjoint(ctx, p, p, p) == -5
    assert L.grmhd_step_adjoint(ctx, None, p, C.c_double(0.1)) == -1
    assert L.grmhd_free(ctx) == 0
    assert L.grmhd_free(None) == -1


def test_adjoint_workspace(lib):
    """The adjoint part of the workspace: FP64 only, ns+1 ghosted stage caches,
    stage flags, five dense arrays (stage state, two U cotangents, the
    right-hand side's cotangent, the pulled-back primitive cotangent), the
    18 face-state cotangents of every axis and the primitive cotangents at
    every axis' ghost positions on top of the forward workspace."""
    L = lib.load()
    n = (16, 8, 6)
    g = lib.make_grid(n, (0, 0, 0), (1, 1, 1), (0, 1, 1))
    for rk in (2, 3):
        o = lib.Opts()
        o.rk_order = rk
        fwd = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
        o.adjoint = 1
        adj = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
        px = ((16 + 4 + 7) // 8) * 8
        sv = px * 12 * 10
        N = 16 * 8 * 6
        nf = 17 * 8 * 6 + 16 * 9 * 6 + 16 * 8 * 7
        ghosts = 4 * (N // 16 + N // 8 + N // 6)   # 4 ghost positions per line and axis
        want = 8 * 9 * ((rk + 1) * sv + 5 * N + ghosts) + rk * N + 8 * 18 * nf
        assert want <= adj - fwd <= want + 256 * 16
        o.precision = 1                      # mixed: no adjoint workspace, and init refuses it
        assert L.grmhd_workspace_bytes(C.byref(g), C.byref(o)) < fwd
    raw, addr = _host_ws(adj)
    m = lib.Metric(lib.FLAT, 0, 0.0, 1.0)
    e = lib.Eos(0, 5.0 / 3.0, 0.0)
    o = lib.Opts(3, 1, 1.0, 1.0, 1e-12, 1e-12, 1e-12, 50, 0, 0, 0, 0, 1, 0, C.c_void_p(addr), adj)
    ctx = C.c_void_p()
    assert L.grmhd_init(C.byref(ctx), C.byref(m), C.byref(g), C.byref(e), C.byref(o)) == -1
    o.precision = 0
    assert L.grmhd_init(C.byref(ctx), C.byref(m), C.byref(g), C.byref(e), C.byref(o)) == 0
    assert L.grmhd_free(ctx) == 0


def test_adjoint_cell_limit(lib):
    """The adjoint kernels index cells, faces and ghost positions in 32 bits:
    an adjoint context holds at most 2^30 cells (a forward one more)."""
    L = lib.load()
    m = lib.Metric(lib.FLAT, 0, 0.0, 1.0)
    e = lib.Eos(0, 5.0 / 3.0, 0.0)
    for n, fits in (((1024, 1024, 1024), True), ((1024, 1024, 1025), False)):
        g = lib.make_grid(n, (0, 0, 0), (1, 1, 1), (0, 0, 0))
        o = lib.Opts()
        fwd = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
        o.adjoint = 1
        adj = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
        assert fwd > 0
        assert (adj > fwd) if fits else (adj == 0)
        o = lib.Opts(3, 0, 1.0, 1.0, 1e-12, 1e-12, 1e-12, 50, 0, 0, 0, 0, 1, 0, None, 0)   # FP64, adjoint
        ctx = C.c_void_p()
        # past the limit the grid is refused before the (missing) workspace is looked at
        rc = L.grmhd_init(C.byref(ctx), C.byref(m), C.byref(g), C.byref(e), C.byref(o))
        assert rc == (-2 if fits else -1)


def test_tape_workspace_and_validation(lib):
    """Tape slots of recorded steps: (rk+1) ghosted FP64 caches and rk flag
    bytes per cell per slot; slot and state checks happen on the host."""
    L = lib.load()
    n = (16, 8, 6)
    g = lib.make_grid(n, (0, 0, 0), (1, 1, 1), (0, 1, 1))
    px = ((16 + 4 + 7) // 8) * 8
    sv = px * 12 * 10
    N = 16 * 8 * 6
    up = lambda x: (x + 255) // 256 * 256
    for rk in (2, 3):
        o = lib.Opts()
        o.rk_order = rk
        o.adjoint = 1
        base = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
        o.tape_steps = 5
        taped = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
        assert taped - base == 5 * ((rk + 1) * up(8 * 9 * sv) + up(rk * N))
        o.adjoint = 0                        # the tape belongs to the adjoint workspace
        assert L.grmhd_workspace_bytes(C.byref(g), C.byref(o)) < base
    o = lib.Opts()
    o.rk_order, o.adjoint, o.tape_steps, o.rho_atm, o.p_atm = 2, 1, 3, 1e-12, 1e-12
    nb = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
    raw, addr = _host_ws(nb)
    o.workspace, o.workspace_bytes = C.c_void_p(addr), nb
    m = lib.Metric(lib.FLAT, 0, 0.0, 1.0)
    e = lib.Eos(0, 5.0 / 3.0, 0.0)
    ctx = C.c_void_p()
    for bad in (-1, 4097):
        o.tape_steps = bad
        assert L.grmhd_init(C.byref(ctx), C.byref(m), C.byref(g), C.byref(e), C.byref(o)) == -1
    o.tape_steps = 3
    assert L.grmhd_init(C.byref(ctx), C.byref(m), C.byref(g), C.byref(e), C.byref(o)) == 0
    dummy = C.c_void_p(addr)                 # never dereferenced: every call below fails its checks
    assert L.grmhd_step_record(ctx, dummy, 0.1, 3) == -1          # slot out of range
    assert L.grmhd_step_record(ctx, dummy, 0.1, -1) == -1
    assert L.grmhd_step_record(ctx, dummy, float("nan"), 0) == -1
    assert L.grmhd_step_record(ctx, dummy, 0.1, 0) == -4          # no primitives yet (cons/prim first)
    assert L.grmhd_step_adjoint_recorded(ctx, 0, dummy) == -4     # slot never recorded
    assert L.grmhd_step_adjoint_recorded(ctx, 3, dummy) == -1
    assert L.grmhd_free(ctx) == 0


def test_ppm_layout_and_validation(lib):
    """PPM widens the ghost layers of the primitive caches from 2 to 3, needs
    3 cells on every active axis and has no adjoint."""
    L = lib.load()
    g = lib.make_grid((16, 8, 6), (0, 0, 0), (1, 1, 1), (0, 1, 1))
    o = lib.Opts()
    o.rk_order = 3
    mc = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
    o.reconstruction = 1
    ppm = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
    sv_mc, sv_ppm = 24 * 12 * 10, 24 * 14 * 12        # x pitch rounded to 8 elements
    assert ppm - mc == 3 * 8 * 9 * (sv_ppm - sv_mc)      # three caches
    o.reconstruction = 2
    assert L.grmhd_workspace_bytes(C.byref(g), C.byref(o)) == 0
    o.reconstruction = 1
    assert L.grmhd_workspace_bytes(C.byref(lib.make_grid((16, 2, 6), (0, 0, 0), (1, 1, 1), (0, 0, 0))),
                                   C.byref(o)) == 0
    assert L.grmhd_workspace_bytes(C.byref(lib.make_grid((16, 1, 1), (0, 0, 0), (1, 1, 1), (0, 0, 0))),
                                   C.byref(o)) > 0
    o.adjoint = 1
    assert L.grmhd_workspace_bytes(C.byref(g), C.byref(o)) == 0
    o.adjoint = 0
    raw, addr = _host_ws(ppm)
    o.workspace, o.workspace_bytes, o.rho_atm, o.p_atm = C.c_void_p(addr), ppm, 1e-12, 1e-12
    m = lib.Metric(lib.FLAT, 0, 0.0, 1.0)
    e = lib.Eos(0, 5.0 / 3.0, 0.0)
    ctx = C.c_void_p()
    assert L.grmhd_init(C.byref(ctx), C.byref(m), C.byref(g), C.byref(e), C.byref(o)) == 0
    assert L.grmhd_free(ctx) == 0
    o.adjoint = 1
    assert L.grmhd_init(C.byref(ctx), C.byref(m), C.byref(g), C.byref(e), C.byref(o)) == -1


def test_fluxct_layout_and_validation(lib):
    """Flux-CT adds the edge values of every pair of active axes to the
    workspace and has no adjoint."""
    L = lib.load()
    for n, pairs in (((16, 8, 6), [(17 * 9 * 6), (17 * 7 * 8), (9 * 7 * 16)]), ((16, 8, 1), [17 * 9]),
                     ((16, 1, 1), [])):
        g = lib.make_grid(n, (0, 0, 0), (1, 1, 1), (0, 1, 1))
        o = lib.Opts()
        o.rk_order = 3
        base = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
        o.divergence = 1
        ct = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
        want = sum(8 * p for p in pairs)
        assert want <= ct - base <= want + 256 * 3, (n, ct - base, want)
        o.divergence = 2
        assert L.grmhd_workspace_bytes(C.byref(g), C.byref(o)) == 0
        o.divergence, o.adjoint = 1, 1
        assert L.grmhd_workspace_bytes(C.byref(g), C.byref(o)) == 0


def test_stored_metric_buffer_and_validation(lib):
    """The stored-metric buffer: 8 centre values per cell and 2 values per face
    of every active axis; host-side checks of grmhd_set_metric and the state
    rule (no cons before the metric is set)."""
    L = lib.load()
    up = lambda x: (x + 255) // 256 * 256
    g = lib.make_grid((16, 8, 6), (0, 0, 0), (1, 1, 1), (0, 1, 1))
    N = 16 * 8 * 6
    want = up(8 * 8 * N) + up(8 * 2 * 17 * 8 * 6) + up(8 * 2 * 16 * 9 * 6) + up(8 * 2 * 16 * 8 * 7)
    assert L.grmhd_metric_bytes(C.byref(g)) == want
    g1 = lib.make_grid((16, 1, 1), (0, 0, 0), (1, 1, 1), (0, 0, 0))
    assert L.grmhd_metric_bytes(C.byref(g1)) == up(8 * 8 * 16) + up(8 * 2 * 17) + 0 + 0
    o = lib.Opts()
    o.rk_order, o.rho_atm, o.p_atm = 3, 1e-12, 1e-12
    nb = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
    raw, addr = _host_ws(nb)
    o.workspace, o.workspace_bytes = C.c_void_p(addr), nb
    e = lib.Eos(0, 5.0 / 3.0, 0.0)
    dummy = C.c_void_p(addr)                 # never dereferenced: every call below fails its checks
    ctx = C.c_void_p()
    assert L.grmhd_init(C.byref(ctx), C.byref(lib.Metric(lib.FLAT, 0, 0.0, 1.0)), C.byref(g), C.byref(e),
                        C.byref(o)) == 0
    assert L.grmhd_set_metric(ctx, dummy, dummy, dummy, 1 << 30) == -1   # not a STORED context
    assert L.grmhd_free(ctx) == 0
    assert L.grmhd_init(C.byref(ctx), C.byref(lib.Metric(lib.STORED, 0, 0.0, 1.0)), C.byref(g), C.byref(e),
                        C.byref(o)) == 0
    assert L.grmhd_cons(ctx, dummy, dummy) == -4                          # metric not set yet
    assert L.grmhd_prim(ctx, dummy, dummy) == -4
    assert L.grmhd_set_metric(ctx, dummy, dummy, dummy, want - 8) == -2   # buffer too small
    assert L.grmhd_set_metric(ctx, dummy, dummy, C.c_void_p(addr + 8), want) == -2
    assert L.grmhd_free(ctx) == 0
    o.adjoint = 1
    nb = L.grmhd_workspace_bytes(C.byref(g), C.byref(o))
    raw2, addr2 = _host_ws(nb)
    o.workspace, o.workspace_bytes = C.c_void_p(addr2), nb
    assert L.grmhd_init(C.byref(ctx), C.byref(lib.Metric(lib.STORED, 0, 0.0, 1.0)), C.byref(g), C.byref(e),
                        C.byref(o)) == -1                                  # no adjoint with a stored metric


def test_batch_workspace_and_init_validation(lib):
    L = lib.load()
    n = [20, 35, 7]
    arrs = ((C.c_int * 3)(*n), (C.c_double * 3)(0, 0, 0), (C.c_double * 3)(1, 1, 1),
            (C.c_double * 3)(0.02, 0.01, 0.05), (C.c_int * 3)(20, 40, 8))
    desc = lib.BatchDesc(3, *arrs, lib.OUTFLOW)
    o = lib.Opts()
    o.rk_order = 3
    nb = L.grmhd_batch_workspace_bytes(C.byref(desc), C.byref(o))
    ncell, nrow = sum(n), sum(9 * (v + 4) for v in n)
    # counters, two record arrays, order, three rows, stage state, tuning state
    assert nb >= 8 * (3 * nrow + 9 * ncell + 9 * ncell)
    o.precision = 1
    assert L.grmhd_batch_workspace_bytes(C.byref(desc), C.byref(o)) < nb
    bad = lib.BatchDesc(3, (C.c_int * 3)(20, 1, 7), *arrs[1:], lib.OUTFLOW)
    assert L.grmhd_batch_workspace_bytes(C.byref(bad), C.byref(o)) == 0
    o.precision = 0
    raw, addr = _host_ws(nb)
    e = lib.Eos(0, 5.0 / 3.0, 0.0)
    o = lib.Opts(3, 0, 1.0, 1.0, 1e-12, 1e-12, 1e-12, 50, 0, 0, 0, 0, 0, 0, C.c_void_p(addr), nb)
    ctx = C.c_void_p()
    assert L.grmhd_batch_init(C.byref(ctx), C.byref(desc), C.byref(e), C.byref(o)) == 0
    assert L.grmhd_batch_evolve(ctx, C.c_void_p(addr), 5) == -4      # before cons
    assert L.grmhd_batch_evolve(ctx, None, 5) == -1
    busy = C.c_double()
    assert L.grmhd_batch_busy(ctx, C.byref(busy), None) == -4         # no evolve launch yet
    assert L.grmhd_batch_busy(ctx, None, None) == -1
    assert L.grmhd_batch_busy(None, C.byref(busy), None) == -1
    assert L.grmhd_batch_tune(ctx, C.c_void_p(addr), 5, None, None) == -4
    assert L.grmhd_batch_set_shape(ctx, 384, 0) == -1
    assert L.grmhd_batch_set_shape(ctx, 1024, 0) == 0
    # rows in LDS need the device to allow their LDS size at init: refused
    # where there is no device
    import torch
    have_gpu = torch.cuda.device_count() > 0
    assert L.grmhd_batch_set_shape(ctx, 1024, 1) == (0 if have_gpu else -1)
    # the split placement: 256 threads only, sized for the device at init
    assert L.grmhd_batch_set_shape(ctx, 512, 2) == -1
    assert L.grmhd_batch_set_shape(ctx, 256, 2) == (0 if have_gpu else -1)
    assert L.grmhd_batch_set_shape(ctx, 256, 3) == -1
    assert L.grmhd_batch_free(ctx) == 0
    o.workspace_bytes = nb - 8
    assert L.grmhd_batch_init(C.byref(ctx), C.byref(desc), C.byref(e), C.byref(o)) == -2


def test_rhs_noalloc_validates_before_touching_a_device(lib):
    """Refusals of grmhd_rhs_noalloc happen host-side, before any HIP call:
    missing arguments, the stored metric (whose buffer would be a second
    allocation), and a grid whose workspace exceeds the static scratch."""
    L = lib.load()
    g = lib.make_grid((16, 8, 4), (0, 0, 0), (1, 1, 1), (0, 0, 0))
    m = lib.Metric(0, 0, 0.0, 1.0)
    e = lib.Eos(0, 5.0 / 3.0, 0.0)
    o = lib.Opts()
    o.rk_order, o.rho_atm = 3, 1e-10
    fake = C.c_void_p(256)   # never dereferenced: every call below is refused first
    ERR_ARG, ERR_WS = -1, -2
    assert L.grmhd_rhs_noalloc(None, C.byref(g), C.byref(e), C.byref(o), fake, fake, None) == ERR_ARG
    assert L.grmhd_rhs_noalloc(C.byref(m), C.byref(g), C.byref(e), C.byref(o), None, fake, None) == ERR_ARG
    stored = lib.Metric(2, 0, 0.0, 1.0)
    assert L.grmhd_rhs_noalloc(C.byref(stored), C.byref(g), C.byref(e), C.byref(o), fake, fake, None) == ERR_ARG
    big = lib.make_grid((64, 64, 64), (0, 0, 0), (1, 1, 1), (0, 0, 0))
    assert L.grmhd_workspace_bytes(C.byref(big), C.byref(o)) > lib.NOALLOC_SCRATCH_BYTES
    assert L.grmhd_rhs_noalloc(C.byref(m), C.byref(big), C.byref(e), C.byref(o), fake, fake, None) == ERR_WS
