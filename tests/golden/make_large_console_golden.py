"""Writes tests/golden/large_console_T1048576.npz: the FP64 streamed oracle's render and adjoint
of the 256-track console (bus tree 32 -> 8 -> 2 -> master, seed 5, T = 2^20) for the seeded
output adjoint synth.output_adjoint(5, n_out, T), i.e. the gradients of sum(dY * Y).

Calls only the oracle (`oracle.streamed`, one node at a time in float64 on the CPU) and the
seeded generators; nothing here comes from the HIP path. Stored (all float64):
  Y_sample   outputs at every 32nd sample [n_out, 2, T/32];  Y_absmax  max |Y| per output row
  dS_rows    the source rows sampled below; dS_sample  their adjoints at every 64th sample;
  dS_absmax  max |dS| over every source
  dP_<type>  the whole parameter gradient of each type present
Run from the repository root:  python tests/golden/make_large_console_golden.py   (about
15 GB of host memory and a few minutes on 8 cores).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import streamed  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "large_console_T1048576.npz")
Y_STRIDE, DS_STRIDE = 32, 64
DS_ROWS = (0, 37, 101, 170, 255)


def main() -> None:
    t0 = time.time()
    w = synth.large_console()
    g = w.graph
    n_out = g.count(synth.OUT)
    dY = synth.output_adjoint(w.seed, n_out, w.T)

    def progress(stage, i, n):
        print(f"  {stage} {i}/{n} nodes, {time.time() - t0:.0f} s", flush=True)

    Y, dS, dP = streamed.render_and_adjoint(g.node_type, g.edges, w.sources, w.params, dY,
                                            progress=progress)
    Y, dS = Y.numpy(), dS.numpy()
    rec = {"T": np.int64(w.T), "seed": np.int64(w.seed), "num_nodes": np.int64(g.num_nodes),
           "Y_stride": np.int64(Y_STRIDE), "dS_stride": np.int64(DS_STRIDE),
           "Y_sample": Y[:, :, ::Y_STRIDE].copy(), "Y_absmax": np.abs(Y).max(axis=(1, 2)),
           "dS_rows": np.array(DS_ROWS, dtype=np.int64),
           "dS_sample": dS[list(DS_ROWS), :, ::DS_STRIDE].copy(),
           "dS_absmax": np.float64(np.abs(dS).max())}
    for t, d in dP.items():
        if d.shape[0] > 0:
            rec[f"dP_{t}"] = d.numpy()
    np.savez_compressed(OUT, **rec)
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1e6:.1f} MB) in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
