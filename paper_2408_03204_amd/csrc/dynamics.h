// Device helpers shared by the dynamics kernels (compressor and noisegate with one ballistics
// constant, k_comp.hip; compressor with attack/release ballistics, k_comp_ar.hip): chunk geometry,
// the static gain curves (paper Eqs. 10-11 and the noisegate of Sec. 3), the chunk ticket and
// publication protocol, and the gather-sum staging of a chunk into LDS.
#pragma once

#include "device_common.h"
#include "kernels.h"

namespace grafx {
namespace dyn {

constexpr int kPer = 12;
constexpr int kChunk = kCompChunk;  // 256 x kPer

// LDS layout of a chunk: element x sits at x + x / 96, one padding word after every 8 threads'
// segments of kPer samples. Thread j's segment is then contiguous from seg_base(j), and the 32
// lanes that one LDS cycle serves, reading element i of their own segments (a 12-word stride
// that would put 4 lanes on each of 8 banks), fall on 32 distinct banks; the coalesced staging
// writes and the stores stay conflict-free.
constexpr int kLdsChunk = kChunk + kChunk / 96;
__device__ __forceinline__ int lpos(int x) { return x + x / 96; }
__device__ __forceinline__ int seg_base(int j) { return kPer * j + (j >> 3); }
static_assert(kPer * 8 == 96, "one padding word per 8 segments");
constexpr double kEps = 1e-8;
constexpr uint64_t kNotReady = ~0ull;

// Coefficient structs passed to the curves provide thr (T), knee (W), c = 1/R - 1 and
// g1 = 1 - R, inv2w = 1/(2W), inv4w = 1/(4W) (0 for a hard knee) and invR2 = 1/R^2.
struct Curve {
  float e, dG, dT, dW, dR;
};

// e = G_y - G_u of the quadratic-knee curve (Eqs. 10-11) and its partial derivatives, without
// branches: the three regions (below the knee, inside it, above it) are selected per lane.
template <bool GRAD, class K>
__device__ __forceinline__ Curve comp_curve(float Gu, const K& k) {
  const float d = Gu - k.thr;
  const float q = d + k.knee;
  const bool soft = k.knee > 0.f;
  const bool below = soft ? (q < 0.f) : (d < 0.f);  // Gu < T - W (soft) or Gu < T (hard)
  const bool knee = soft && !below && d < k.knee;   // T - W <= Gu < T + W
  Curve o;
  const float e_knee = k.c * q * q * k.inv4w, e_lin = k.c * d;
  o.e = below ? 0.f : (knee ? e_knee : e_lin);
  if (GRAD) {
    const float g_knee = k.c * q * k.inv2w;
    o.dG = below ? 0.f : (knee ? g_knee : k.c);
    o.dT = -o.dG;
    const float w_knee = k.c * (q * k.inv2w - q * q * k.inv4w * (2.f * k.inv2w));
    o.dW = knee ? w_knee : 0.f;
    const float r_knee = -q * q * k.inv4w * k.invR2, r_lin = -d * k.invR2;
    o.dR = below ? 0.f : (knee ? r_knee : r_lin);
  } else {
    o.dG = o.dT = o.dW = o.dR = 0.f;
  }
  return o;
}

// Noisegate curve (Sec. 3 "Noisegate"): e = 0 at or above T + W, (1 - R)(G_u - T - W)^2 / (4W) on
// the knee, (R - 1)(G_u - T) below T - W (hard knee at T when W <= 0), and its derivatives.
template <bool GRAD, class K>
__device__ __forceinline__ Curve gate_curve(float Gu, const K& k) {
  const float d = Gu - k.thr;
  const float q = d - k.knee;  // G_u - T - W
  const bool soft = k.knee > 0.f;
  const bool below = soft ? (d + k.knee < 0.f) : (d < 0.f);  // Gu < T - W (soft) or Gu < T
  const bool knee = soft && !below && q < 0.f;               // T - W <= Gu < T + W
  Curve o;
  const float e_knee = k.g1 * q * q * k.inv4w, e_lin = -k.g1 * d;
  o.e = below ? e_lin : (knee ? e_knee : 0.f);
  if (GRAD) {
    const float g_knee = k.g1 * q * k.inv2w;
    o.dG = below ? -k.g1 : (knee ? g_knee : 0.f);
    o.dT = -o.dG;
    const float w_knee = -k.g1 * (q * k.inv2w + q * q * k.inv4w * (2.f * k.inv2w));
    o.dW = knee ? w_knee : 0.f;
    const float r_knee = -q * q * k.inv4w;
    o.dR = below ? d : (knee ? r_knee : 0.f);
  } else {
    o.dG = o.dT = o.dW = o.dR = 0.f;
  }
  return o;
}

// ln x and exp x through the hardware base-2 instructions (v_log_f32, v_exp_f32). x > 0 is
// normal here (the envelope plus 1e-8); the exp argument is a gain in natural-log units, whose
// relative error grows with its magnitude (about 2e-6 at |x| = 30).
__device__ __forceinline__ float ln_f(float x) {
  return __builtin_amdgcn_logf(x) * 0.69314718055994531f;
}
__device__ __forceinline__ float exp_f(float x) {
  return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
}

__device__ __forceinline__ int comp_chunks_of(int64_t n) { return (int)((n + kChunk - 1) / kChunk); }

// Node of a block within its step: a node's `chunks` blocks contiguous (order 0) or the step's
// nodes interleaved block by block (order 1). A block's chunk comes from its node's ticket, so
// the order decides only when a node's chunks are issued, not what they compute.
__device__ __forceinline__ int block_node(const GraphView& g, int n_nodes, int chunks) {
  return g.dyn_order ? (int)blockIdx.x % n_nodes : (int)blockIdx.x / chunks;
}

// ---- chunk chaining ---------------------------------------------------------------------------

__device__ __forceinline__ int take_ticket(unsigned* counter, int* sh) {
  __syncthreads();
  if (threadIdx.x == 0)
    *sh = (int)__hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return *sh;
}

__device__ __forceinline__ void publish(uint64_t* slot, double v) {
  __hip_atomic_store(slot, (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Wait for a published total: at most `polls` reads of the slot (0: give up at once). A wait
// that gives up sets bit 0 of the error word and returns NaN, so the kernel still ends normally.
__device__ __forceinline__ double await_total(uint64_t* slot, unsigned* err, int polls) {
  for (int spin = 0; spin < polls; ++spin) {
    const uint64_t x = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (x != kNotReady) return __longlong_as_double((long long)x);
    __builtin_amdgcn_s_sleep(1);
  }
  atomicOr(err, 1u);
  return __longlong_as_double(0x7FF8000000000001ll);
}

// ---- staging -----------------------------------------------------------------------------------

// Gather-sum of a chunk (both channels) into LDS (padded layout): ADJ = false sums the input
// edges over U/S, ADJ = true the output edges over dU/dY. Zero beyond T.
template <bool ADJ, bool RAGGED>
__device__ __forceinline__ void stage(const GraphView& g, int node, int t0, float* sl, float* sr) {
  const int64_t T = g.T;
  const int e0 = ADJ ? g.out_ptr[node] : g.in_ptr[node];
  const int e1 = ADJ ? g.out_ptr[node + 1] : g.in_ptr[node + 1];
  float l[kPer], r[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) l[q] = r[q] = 0.f;
  for (int e = e0; e < e1; ++e) {  // all loads of a row issued before any is consumed
    const int other = ADJ ? g.out_dst[e] : g.in_src[e];
    const float* row = ADJ ? adj_row(g, other) : out_row(g, other);
    const int64_t L = RAGGED ? (int64_t)g.len[other] : T;
    const auto rl = row_rsrc(row, L), rr = row_rsrc(row + T, L);
    float xl[kPer], xr[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = t0 + (int)threadIdx.x + kBlock * q;
      xl[q] = bload_nt(rl, t);
      xr[q] = bload_nt(rr, t);
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      l[q] += xl[q];
      r[q] += xr[q];
    }
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    sl[lpos(threadIdx.x + kBlock * q)] = l[q];
    sr[lpos(threadIdx.x + kBlock * q)] = r[q];
  }
}

// x = (u_l + u_r)^2 at LDS position idx, formed in float and fed to the double envelope
// recursion.
__device__ __forceinline__ double energy(const float* sl, const float* sr, int idx) {
  const float m = sl[idx] + sr[idx];
  return (double)(m * m);
}

// Chunk store (from the padded layout) into a row of stride T; samples at or beyond the node's
// length Tn are dropped.
__device__ __forceinline__ void store_chunk(float* row, int64_t T, int64_t Tn, int t0,
                                            const float* sl, const float* sr) {
  const auto rl = row_rsrc(row, Tn), rr = row_rsrc(row + T, Tn);
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    // an opaque copy of the thread index keeps the compiler from holding the staging
    // addresses, which are the same, in registers from the staging to here
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int idx = tid + kBlock * q;
    bstore_nt(rl, t0 + idx, sl[lpos(idx)]);
    bstore_nt(rr, t0 + idx, sr[lpos(idx)]);
  }
}

}  // namespace dyn
}  // namespace grafx
