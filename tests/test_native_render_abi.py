"""Argument checking of the render entry points of the C ABI (grafx_render,
grafx_render_backward, the single-step calls, grafx_workspace_error), called through ctypes with
fake device addresses. Every call here must be refused during validation, which runs before any
HIP call: a failed call enqueues nothing, so these tests need no GPU (a call that got past its
checks would touch the fake addresses and could not pass on this host).

Error model (the boundary's own; the paper has none): NULL handle or buffer -> GRAFX_E_ARG,
T out of range / misaligned buffer / missing parameter tensor -> GRAFX_E_SHAPE, workspace too
small -> GRAFX_E_WORKSPACE, step out of range -> GRAFX_E_ARG."""
import ctypes

import pytest

import synth
from paper_2408_03204_amd import Schedule, load
from paper_2408_03204_amd import _lib

OK, E_ARG, E_SHAPE, E_WORKSPACE = 0, 1, 5, 7
BASE = 1 << 40  # fake, 256-byte aligned device addresses (never dereferenced)


def addr(i: int, misalign: int = 0) -> int:
    return BASE + i * (1 << 32) + misalign


@pytest.fixture(scope="module")
def console():
    w = synth.tiny_console(T=8)  # gain_pan, eq, compressor, mix, out
    return Schedule(w.graph.node_type, w.graph.edges)


def params(sched, skip=None):
    arr = _lib.ptr_array()
    for t in range(_lib.NUM_TYPES):
        if sched.type_count[t] and t != skip and t in (3, 4, 5, 6, 7, 8, 9, 10, 11, 12):
            arr[t] = addr(10 + t)
    return arr


def ws_bytes(sched, T, bwd):
    return sched.workspace_bytes(T if 1 <= T < (1 << 29) else 4096, bwd)


def render(sched, T=4096, plan=None, S=None, P=None, U=None, ws=None, nbytes=None, h=True):
    lib = load()
    return lib.grafx_render(
        sched._h if h else None, addr(1) if plan is None else plan, T,
        addr(2) if S is None else S, params(sched) if P is None else P,
        addr(3) if U is None else U, addr(4) if ws is None else ws,
        ws_bytes(sched, T, False) if nbytes is None else nbytes, None)


def backward(sched, T=4096, dY=None, dU=None, dS=0, ws=None, nbytes=None, U=None):
    lib = load()
    return lib.grafx_render_backward(
        sched._h, addr(1), T, addr(2), params(sched), addr(3) if U is None else U,
        addr(5) if dY is None else dY, addr(6) if dU is None else dU, dS or None,
        _lib.ptr_array(), addr(4) if ws is None else ws,
        ws_bytes(sched, T, True) if nbytes is None else nbytes, None)


def err():
    return load().grafx_last_error().decode()


def test_render_rejects_bad_arguments(console):
    s = console
    assert render(s, h=False) == E_ARG and "schedule" in err()
    assert render(s, plan=0) == E_ARG and "plan" in err()
    assert render(s, T=0) == E_SHAPE
    assert render(s, T=1 << 29) == E_SHAPE
    assert render(s, U=0) == E_ARG and "U" in err()
    assert render(s, S=0) == E_ARG and "S" in err()
    assert render(s, plan=addr(1, 4)) == E_SHAPE and "aligned" in err()
    assert render(s, U=addr(3, 4)) == E_SHAPE and "aligned" in err()
    assert render(s, S=addr(2, 8)) == E_SHAPE
    assert render(s, ws=addr(4, 16)) == E_SHAPE and "workspace" in err()
    for t in (3, 4, 5):  # a parameter tensor of a type the graph uses is missing
        assert render(s, P=params(s, skip=t)) == E_SHAPE and str(t) in err()
    need = ws_bytes(s, 4096, False)
    assert need > 0
    assert render(s, nbytes=need - 1) == E_WORKSPACE and str(need) in err()
    assert render(s, ws=0, nbytes=need) == E_WORKSPACE


def test_workspace_size_depends_on_T(console):
    s = console
    small = ws_bytes(s, 4096, False)
    assert render(s, T=1 << 20, nbytes=small) == E_WORKSPACE


def test_backward_rejects_bad_arguments(console):
    s = console
    assert backward(s, dY=0) == E_ARG
    assert backward(s, dU=0) == E_ARG
    assert backward(s, dU=addr(6, 4)) == E_SHAPE
    assert backward(s, dY=addr(5, 12)) == E_SHAPE
    assert backward(s, dS=addr(7, 4)) == E_SHAPE
    # a workspace sized for the forward call only is too small for the adjoint
    fwd = ws_bytes(s, 4096, False)
    assert fwd < ws_bytes(s, 4096, True)
    assert backward(s, nbytes=fwd) == E_WORKSPACE
    assert backward(s, U=0) == E_ARG


def test_single_steps_reject_out_of_range_steps(console):
    s, lib, T = console, load(), 4096
    for step in (0, -1, s.num_steps + 1):
        r = lib.grafx_render_step(s._h, addr(1), T, addr(2), params(s), addr(3), addr(4),
                                  ws_bytes(s, T, False), step, None)
        assert r == E_ARG and "step" in err()
    for step in (0, s.num_steps):  # the output step has no adjoint of its own
        r = lib.grafx_render_backward_step(s._h, addr(1), T, addr(2), params(s), addr(3),
                                           addr(5), addr(6), addr(4), ws_bytes(s, T, True),
                                           step, None)
        assert r == E_ARG and "step" in err()


def test_workspace_error_query_rejects_bad_arguments(console):
    s, lib, T = console, load(), 4096
    word = ctypes.c_uint32(7)
    p = ctypes.addressof(word)
    assert lib.grafx_workspace_error(None, T, addr(4), ws_bytes(s, T, False), p, None) == E_ARG
    assert lib.grafx_workspace_error(s._h, T, None, ws_bytes(s, T, False), p, None) == E_ARG
    assert lib.grafx_workspace_error(s._h, T, addr(4), ws_bytes(s, T, False), None, None) == E_ARG
    assert lib.grafx_workspace_error(s._h, 0, addr(4), ws_bytes(s, T, False), p, None) == E_SHAPE
    assert lib.grafx_workspace_error(s._h, T, addr(4, 8), ws_bytes(s, T, False), p,
                                     None) == E_SHAPE
    assert lib.grafx_workspace_error(s._h, T, addr(4), 16, p, None) == E_WORKSPACE
    assert word.value == 7  # nothing was written


def test_plan_upload_rejects_bad_arguments(console):
    s, lib = console, load()
    assert lib.grafx_plan_upload(None, addr(1), s.plan_bytes, None) == E_ARG
    assert lib.grafx_plan_upload(s._h, None, s.plan_bytes, None) == E_ARG
    assert lib.grafx_plan_upload(s._h, addr(1), s.plan_bytes - 1, None) == E_WORKSPACE
    assert lib.grafx_plan_upload(s._h, addr(1, 4), s.plan_bytes, None) == E_SHAPE


def noalloc(sched, T=4096, plan=None, S=None, P=None, U=None, h=True):
    return load().grafx_render_noalloc(
        sched._h if h else None, addr(1) if plan is None else plan, T,
        addr(2) if S is None else S, params(sched) if P is None else P,
        addr(3) if U is None else U, None)


def test_noalloc_render_rejects_bad_arguments(console):
    assert noalloc(console, h=False) == E_ARG
    assert noalloc(console, plan=0) == E_ARG
    assert noalloc(console, U=0) == E_ARG
    assert noalloc(console, T=0) == E_SHAPE
    assert noalloc(console, T=1 << 29) == E_SHAPE
    assert noalloc(console, plan=addr(1, 128)) == E_SHAPE
    assert noalloc(console, U=addr(3, 4)) == E_SHAPE
    assert noalloc(console, P=params(console, skip=4)) == E_SHAPE


def test_noalloc_render_refuses_a_workspace_beyond_its_scratch():
    """A render whose forward workspace exceeds the static scratch (32 MiB) fails with
    GRAFX_E_WORKSPACE during validation, before any HIP call."""
    b = synth.GraphBuilder()
    i0, m = b.add(synth.IN), b.add(synth.MIX)
    for _ in range(48):
        c = b.add(synth.COMP)
        b.connect(i0, c)
        b.connect(c, m)
    b.connect(m, b.add(synth.OUT))
    g = b.build()
    sched = Schedule(g.node_type, g.edges)
    T = 1 << 28
    assert sched.workspace_bytes(T, False) > (32 << 20)
    assert noalloc(sched, T=T) == E_WORKSPACE
    assert b"static scratch" in load().grafx_last_error()
    # within the scratch the same graph passes validation and only then needs a device: on a host
    # without one the call fails at the scratch lookup (GRAFX_E_HIP), having launched nothing
    small = 1 << 16
    assert sched.workspace_bytes(small, False) <= (32 << 20)
    if not _has_device():
        assert noalloc(sched, T=small) == 8  # GRAFX_E_HIP
        assert b"scratch address" in load().grafx_last_error()


def _has_device() -> bool:
    import torch
    return torch.cuda.device_count() > 0


@pytest.fixture(scope="module")
def reverb_sched():
    b = synth.GraphBuilder()
    i0 = b.add(synth.IN)
    r = b.add(synth.REVERB)
    b.connect(i0, r)
    b.connect(r, b.add(synth.OUT))
    g = b.build()
    return Schedule(g.node_type, g.edges)


def test_reverb_needs_its_noise(reverb_sched):
    """A graph with reverb nodes renders only once a noise realisation is set; the noise length
    is the FIR length and enters the workspace size; bad settings are refused."""
    s = reverb_sched
    lib = load()
    assert s.type_count[synth.REVERB] == 1
    assert lib.grafx_schedule_set_reverb_noise(s._h, None, 0) == OK
    assert render(s) == E_ARG and "noise" in err()
    assert lib.grafx_schedule_set_reverb_noise(None, addr(9), 100) == E_ARG
    assert lib.grafx_schedule_set_reverb_noise(s._h, None, 100) == E_ARG
    assert lib.grafx_schedule_set_reverb_noise(s._h, addr(9), 0) == E_SHAPE
    assert lib.grafx_schedule_set_reverb_noise(s._h, addr(9), (1 << 22) + 1) == E_SHAPE
    assert lib.grafx_schedule_set_reverb_noise(s._h, addr(9, 2), 100) == E_SHAPE
    assert lib.grafx_schedule_set_reverb_noise(s._h, addr(9), 4000) == OK
    short_ws = s.workspace_bytes(4096, True)
    assert lib.grafx_schedule_set_reverb_noise(s._h, addr(9), 88200) == OK
    long_ws = s.workspace_bytes(4096, True)
    assert long_ws > short_ws
    # with the noise set, the remaining checks are the render's own
    assert render(s, P=params(s, skip=synth.REVERB)) == E_SHAPE and "11" in err()
    assert render(s, nbytes=long_ws // 4) == E_WORKSPACE
    assert lib.grafx_schedule_set_reverb_noise(s._h, None, 0) == OK


def test_delay_surrogate_setting():
    """The delay-time surrogate is off by default; turning it on grows the adjoint's workspace
    (spectra and correlation of every delay node) and leaves the forward workspace alone."""
    b = synth.GraphBuilder()
    i0 = b.add(synth.IN)
    d = b.add(synth.DELAY)
    b.connect(i0, d)
    b.connect(d, b.add(synth.OUT))
    g = b.build()
    s = Schedule(g.node_type, g.edges)
    lib = load()
    fwd, bwd = s.workspace_bytes(1 << 16, False), s.workspace_bytes(1 << 16, True)
    assert lib.grafx_schedule_set_delay_surrogate(None, 1) == E_ARG
    assert lib.grafx_schedule_set_delay_surrogate(s._h, 2) == E_ARG
    assert lib.grafx_schedule_set_delay_surrogate(s._h, 1) == OK
    assert s.workspace_bytes(1 << 16, False) == fwd
    assert s.workspace_bytes(1 << 16, True) > bwd
    s.set_delay_surrogate(False)
    assert s.workspace_bytes(1 << 16, True) == bwd


def test_delay_phasor_regularise_rejects_bad_arguments():
    lib = load()
    f = lib.grafx_delay_phasor_regularise
    assert f(4, 1, addr(1), addr(2), 1.0, None) == 4  # GRAFX_E_TYPE: not a delay type
    assert f(7, -1, addr(1), addr(2), 1.0, None) == E_SHAPE
    assert f(7, 1, None, addr(2), 1.0, None) == E_ARG
    assert f(12, 1, addr(1), None, 1.0, None) == E_ARG
    assert f(7, 1, addr(1), addr(2), -1.0, None) == E_ARG
    assert f(7, 1, addr(1), addr(2), float("nan"), None) == E_ARG
    assert f(7, 1, addr(1, 2), addr(2), 1.0, None) == E_SHAPE
    assert f(7, 0, None, None, 0.0, None) in (OK, 8)  # nothing to do (no launch needed)
