"""FP64 CPU oracle for the batched audio-graph render and its adjoint (GRAFX, arXiv 2408.03204).

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, calls or links this package;
only the tests, the smoke check and the benchmark's CPU-baseline leg do. It is plain, slow and
written to be checked against the paper by eye:

* `schedule`  -- the type scheduler (Sec. 2 "Type scheduling", Algorithm 1 preprocessing):
                 one-by-one, greedy, beam and optimal schedules, the node reordering, the
                 read/write index lists.
* `processors` -- each differentiable processor (Sec. 3, Eqs. 2-5, 8-12, 14) plus tanh
                 distortion, in torch float64.
* `reverb`    -- the filtered-noise mid/side reverb (Sec. 3, Eqs. 6-7) and the delay-time
                 surrogate with its straight-through gradient (Eq. 15).
* `render`    -- the graph evaluated one node at a time in topological order (Sec. 2,
                 "Definitions", Eq. 1).
* `mrstft`    -- the multi-resolution STFT loss used to drive gradient descent (Sec. 4).
* `encoder`   -- the learned parameter initialiser of the gradient-descent application: log-mel
                 features, the convolutional encoder, its training loss and Adam.

Gradients come from torch autograd in float64. The oracle shares no code with the HIP library.
Parity status of every function is listed in the module that defines it; the only function
without an independent pin is marked "parity unpinned" there.
"""
from . import encoder, mrstft, processors, render, reverb, schedule  # noqa: F401
