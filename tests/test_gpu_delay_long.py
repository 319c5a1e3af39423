"""GPU parity of the 2 s multitap delay (paper Sec. 3 "Multitap delay", Eq. 14 with M = 20 slots of
100 ms, 880 parameters; node type delay_long) against the FP64 oracle: output, source adjoint,
filter-magnitude gradients and, with the surrogate setting on, the straight-through phasor
gradients (Eq. 15). Lengths: a signal that reaches every slot (T = 2^17, four tap-gradient
groups), a ragged one just past 2 s, and one that ends inside slot 6, so that the later slots'
delays fall past the end. Graphs hold 2 s delays in parallel and in series next to a 500 ms one.
Tolerances as for every render: 1e-5 of the peak output, 1e-3 of each parameter column's largest
entry (a phasor's two coordinates judged as one 2-vector)."""
import pytest

import synth
from gpu_common import say
from test_gpu_delay_surrogate import check, run

pytestmark = pytest.mark.gpu


def long_delay_graph(T, seed, off_circle=0.0):
    b = synth.GraphBuilder()
    i0, i1 = b.add(synth.IN), b.add(synth.IN)
    d0, d1, d2 = (b.add(synth.DELAY_LONG) for _ in range(3))
    s0 = b.add(synth.DELAY)
    o = b.add(synth.OUT)
    for s, d in ((i0, d0), (i1, d1), (d1, d2), (i0, s0), (i1, s0), (d0, o), (d2, o), (s0, o)):
        b.connect(s, d)
    g = b.build()
    P = synth.draw_params(synth.rng_for(seed, 2), g)
    if off_circle:
        for t in (synth.DELAY, synth.DELAY_LONG):
            q = P[t].reshape(P[t].shape[0], 2, -1, 22)
            r = 1.0 + off_circle * synth.rng_for(seed, 3 + t).uniform(-1.0, 1.0,
                                                                       size=q.shape[:3] + (1,))
            q[..., :2] *= r.astype(q.dtype)
    return synth.Workload("long_delay_graph", g, synth.make_sources(synth.rng_for(seed, 1), 2, T),
                          P, None, T, seed)


@pytest.mark.parametrize("T,surrogate", [(2 ** 17, False), (2 ** 17, True),
                                         (88200 + 2048 + 777, True), (6 * 4410 + 1234, True)])
def test_long_delay(T, surrogate):
    say(f"[delay 2 s] T={T} surrogate={surrogate}")
    w = long_delay_graph(T, 91, 1e-4 if surrogate else 0.0)
    errs, _, _ = run(w, 9, surrogate=surrogate)
    check(errs)


def test_long_delay_at_the_largest_length():
    T = 2 ** 20
    say(f"[delay 2 s, 2^20] T={T}")
    w = long_delay_graph(T, 92, 1e-4)
    errs, _, _ = run(w, 10, surrogate=True)
    check(errs)
