// The 4096-point complex FFT of 256 threads x 16 points in registers (radix-16 Stockham, two
// LDS transposes) and the windowed gather-sum of a node's inputs or output adjoints, shared by
// the EQ and the reverb kernels.
#pragma once

#include "device_common.h"
#include "kernels.h"
#include "tables.inc"

namespace grafx {
namespace fft4 {

constexpr int kN = kEqFFT;  // 4096
constexpr int kLds = kN + kN / 16;  // one pad slot per 16 entries

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// Twiddles of the two twiddled passes for thread j (the inverse uses their conjugates):
// w1[r] = exp(-2 pi i r (j mod 16) / 256) comes from a 16 x 16 table in LDS, row (j mod 16)
// padded to 17 entries so that the 16 rows read at one r fall in distinct banks; w2[r] =
// exp(-2 pi i r j / 4096) differs in every thread and is kept in registers for all transforms
// of the block.
constexpr int kW1Row = 17;
constexpr int kW1Lds = 16 * kW1Row;

struct Twiddles {
  float2 w2[16];
  const float2* w1;  // LDS table, entry (m, r) at m * kW1Row + r
};

// Fills the LDS table (thread j writes entry (j / 16, j mod 16)) and loads w2; the table is read
// only after the first barrier of the first transform.
__device__ __forceinline__ void load_twiddles(Twiddles& tw, float2* w1lds) {
  const int j = threadIdx.x;
  w1lds[(j >> 4) * kW1Row + (j & 15)] = kTw4096[(j & 15) * (j >> 4) * 16];
#pragma unroll
  for (int r = 1; r < 16; ++r) tw.w2[r] = kTw4096[r * j];
  tw.w1 = w1lds;
}

// In-place 4096-point DFT (forward: exp(-2 pi i nk/N); inverse: exp(+...), unnormalised).
// On entry v[r] holds x[j + 256 r] for thread j; on exit v[r] holds X[j + 256 r]. Bit r of LIVE
// clear states that v[r] is zero on entry in every thread (a zero-padded window), which the first
// pass skips.
template <bool INV, unsigned LIVE = 0xFFFFu>
__device__ __forceinline__ void fft4096(float2 (&v)[16], float2* lds, const Twiddles& tw) {
  const int j = threadIdx.x;
  // The padded index pad(i) of the three access patterns splits into a per-thread base and a
  // multiple of r known at compile time (an immediate offset of the LDS instruction):
  // pad(16 j + r) = 17 j + r, pad(j + 256 r) = j + j / 16 + 272 r and
  // pad(256 (j / 16) + j mod 16 + 16 r) = 272 (j / 16) + j mod 16 + 17 r.
  float2* const l0 = lds + 17 * j;
  float2* const l1 = lds + j + (j >> 4);
  float2* const l2 = lds + (j >> 4) * 272 + (j & 15);
  // pass 0 (sub-transform size 1): no twiddles
  dft16<INV, LIVE>(v);
#pragma unroll
  for (int r = 0; r < 16; ++r) l0[r] = v[r];
  __syncthreads();
  // pass 1 (sub-transform size 16)
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = l1[272 * r];
  const float2* w1 = tw.w1 + (j & 15) * kW1Row;
#pragma unroll
  for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], INV ? cconj(w1[r]) : w1[r]);
  dft16<INV>(v);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) l2[17 * r] = v[r];
  __syncthreads();
  // pass 2 (sub-transform size 256): outputs land at j + 256 r
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = l1[272 * r];
#pragma unroll
  for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], INV ? cconj(tw.w2[r]) : tw.w2[r]);
  dft16<INV>(v);
  __syncthreads();
}

// v[r] = sum over the node's rows of x[w0 + j + 256 r] for r in [r_lo, r_hi) (both channels as
// re/im), zero elsewhere and outside [0, length of the row's node). All loads of one row are
// issued before they are consumed, so a tile waits for memory once per row, not once per load.
template <bool ADJ>
__device__ __forceinline__ void gather_window(const GraphView& g, int node, int w0, float2 (&v)[16],
                                              int r_lo, int r_hi) {
  const int64_t T = g.T;
  const int e0 = ADJ ? g.out_ptr[node] : g.in_ptr[node];
  const int e1 = ADJ ? g.out_ptr[node + 1] : g.in_ptr[node + 1];
  const int j = threadIdx.x;
  auto load_row = [&](int e, float2 (&x)[16]) {
    // the edge, its row and the row's length are the same in every lane: keep them scalar
    const int other = __builtin_amdgcn_readfirstlane(ADJ ? g.out_dst[e] : g.in_src[e]);
    const float* row = ADJ ? adj_row(g, other) : out_row(g, other);
    const int L = __builtin_amdgcn_readfirstlane((int)node_len(g, other));
    const auto rl = row_rsrc(row, L), rr = row_rsrc(row + T, L);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int t = w0 + j + 256 * r;
      x[r] = (r < r_lo || r >= r_hi) ? make_float2(0.f, 0.f)
                                     : make_float2(bload(rl, t), bload(rr, t));
    }
  };
  if (e0 == e1) {  // no incoming rows
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = make_float2(0.f, 0.f);
    return;
  }
  load_row(e0, v);  // the first row is loaded in place, later rows are added to it
  for (int e = e0 + 1; e < e1; ++e) {
    float2 x[16];
    load_row(e, x);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = cadd(v[r], x[r]);
  }
}

}  // namespace fft4
}  // namespace grafx
