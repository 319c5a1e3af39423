// Device-side helpers shared by the kernels: graph gather-sums, block reductions, the
// XCD-aware block order, complex arithmetic and the small in-register DFTs used by the LDS FFTs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace grafx {

constexpr int kBlock = 256;  // threads per block for every streaming kernel (4 wave64)

// Read-side view of the graph for one launch (one schedule step or one adjoint step).
struct GraphView {
  const int32_t* in_ptr;     // [V+1]
  const int32_t* in_src;     // [E]
  const int32_t* out_ptr;    // [V+1]
  const int32_t* out_dst;    // [E]
  const int32_t* param_row;  // [V]
  const float* S;            // [K][2][T] sources
  const float* U;            // [V][2][T] node outputs (rows >= K)
  const float* dY;           // [n_out][2][T] output adjoint
  const float* dU;           // [V][2][T] input adjoints (rows of processed nodes)
  const int32_t* len;        // [V] per-node signal length, or null when every node has length T
  int64_t T;                 // row stride (and the length of every node when len is null)
  int32_t K;                 // number of input nodes (= sigma positions [0, K))
  int32_t out_begin;         // sigma position of the first output node
  int32_t vec4;              // T and every node length are multiples of 4 (16-byte vectors)
  int32_t pw_unroll;         // pointwise kernels: 1024-sample parts per block (1, 2 or 4)
  int32_t wait_polls;        // dynamics kernels: reads of a published chunk state before giving up
  int32_t eq_order;          // EQ kernels: 0 tiles of a node on one XCD, 1 hardware block order
  int32_t dyn_order;         // dynamics kernels: 0 a node's blocks contiguous, 1 nodes interleaved
  int32_t tap_tiles;         // delay tap gradients: tiles per block (4, 8 or 16)
};

// Length of the signal of the node at sigma position v (its row holds valid samples [0, len)).
__device__ __forceinline__ int64_t node_len(const GraphView& g, int v) {
  return g.len ? (int64_t)g.len[v] : g.T;
}

// Row (stereo, [2][T]) holding the output of the node at sigma position s.
__device__ __forceinline__ const float* out_row(const GraphView& g, int s) {
  return s < g.K ? g.S + (int64_t)s * 2 * g.T : g.U + (int64_t)s * 2 * g.T;
}

// Row holding the adjoint of the aggregated input of the node at sigma position d.
__device__ __forceinline__ const float* adj_row(const GraphView& g, int d) {
  return d >= g.out_begin ? g.dY + (int64_t)(d - g.out_begin) * 2 * g.T
                          : g.dU + (int64_t)d * 2 * g.T;
}

// Raw buffer resource over n floats starting at p: loads through it take a 32-bit element
// offset and return 0 outside [0, n) (the hardware range check), which implements the zero
// padding of signal windows without branches. Requires n < 2^29.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float* p, int64_t n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, (int)(n * 4),
                                           0x00020000);
}

__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int idx) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4, 0, 0));
}

// The same load marked non-temporal (cache policy bit 1), for rows read once.
__device__ __forceinline__ float bload_nt(__amdgpu_buffer_rsrc_t r, int idx) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4, 0, 2));
}

// Raw buffer store: an element index outside the resource's range is dropped by the hardware.
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, int idx, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, idx * 4, 0, 0);
}

// The same store marked non-temporal (cache policy bit 1): for the signal rows a step writes,
// which only later steps read back, after the caches have turned over.
__device__ __forceinline__ void bstore_nt(__amdgpu_buffer_rsrc_t r, int idx, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, idx * 4, 0, 2);
}

// A plain non-temporal store of one float.
__device__ __forceinline__ void store_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }

// Blocks are dispatched round-robin over the 8 XCDs of an MI355X; remap the hardware block id so
// that every XCD works through one contiguous range of logical blocks (neighbouring time tiles
// of a node then share an L2, which serves their overlapping halos).
__device__ __forceinline__ int xcd_logical_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, k = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// ---- reductions (fixed tree order: deterministic) ----------------------------------------

template <typename F>
__device__ __forceinline__ F wave_sum(F v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block (kBlock threads); result valid in every thread. `scratch` holds >= 4 F.
template <typename F>
__device__ __forceinline__ F block_sum(F v, F* scratch) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[w] = v;
  __syncthreads();
  F s = scratch[0];
#pragma unroll
  for (int i = 1; i < kBlock / 64; ++i) s += scratch[i];
  return s;
}

// ---- complex helpers -----------------------------------------------------------------------

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---- small DFTs in registers: X[k] = sum_n x[n] exp(-+2 pi i n k / R), natural order --------

template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const float2 t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// exp(-+2 pi i m / 16) for the internal twiddles of the radix-16 DFT
template <bool INV>
__device__ __forceinline__ float2 w16(int m) {
  constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508977f, r2 = 0.70710678118654752f;
  float2 w;
  switch (m & 15) {
    case 0: w = make_float2(1.f, 0.f); break;
    case 1: w = make_float2(c1, -s1); break;
    case 2: w = make_float2(r2, -r2); break;
    case 3: w = make_float2(s1, -c1); break;
    case 4: w = make_float2(0.f, -1.f); break;
    case 6: w = make_float2(-r2, -r2); break;
    case 9: w = make_float2(-c1, s1); break;
    default: w = make_float2(1.f, 0.f); break;  // not used
  }
  return INV ? cconj(w) : w;
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
  // 8 = 2 x 4: n = 2 n1 + n2, k = k1 + 4 k2
  dft4<INV>(v[0], v[2], v[4], v[6]);
  dft4<INV>(v[1], v[3], v[5], v[7]);
  // twiddle w8^(n2 k1) = w16^(2 n2 k1) for n2 = 1
  v[3] = cmul(v[3], w16<INV>(2));
  v[5] = mul_mi<INV>(v[5]);
  v[7] = cmul(v[7], w16<INV>(6));
  float2 o[8];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a = v[2 * k1], b = v[2 * k1 + 1];
    dft2<INV>(a, b);
    o[k1] = a;
    o[k1 + 4] = b;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = o[i];
}

// x + y and x - y where ZX / ZY state that x / y is known to be zero, so no instruction is spent
// on it (the result equals the full sum up to the sign of an exact zero)
template <bool ZX, bool ZY>
__device__ __forceinline__ float2 cadd_z(float2 x, float2 y) {
  if constexpr (ZX && ZY) return make_float2(0.f, 0.f);
  else if constexpr (ZX) return y;
  else if constexpr (ZY) return x;
  else return cadd(x, y);
}
template <bool ZX, bool ZY>
__device__ __forceinline__ float2 csub_z(float2 x, float2 y) {
  if constexpr (ZX && ZY) return make_float2(0.f, 0.f);
  else if constexpr (ZX) return make_float2(-y.x, -y.y);
  else if constexpr (ZY) return x;
  else return csub(x, y);
}

// dft4 whose inputs a_i are known to be zero where Z_i
template <bool INV, bool Z0, bool Z1, bool Z2, bool Z3>
__device__ __forceinline__ void dft4_z(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd_z<Z0, Z2>(a0, a2), t1 = csub_z<Z0, Z2>(a0, a2);
  const float2 t2 = cadd_z<Z1, Z3>(a1, a3), t3 = mul_mi<INV>(csub_z<Z1, Z3>(a1, a3));
  constexpr bool ZE = Z0 && Z2, ZO = Z1 && Z3;
  a0 = cadd_z<ZE, ZO>(t0, t2);
  a2 = csub_z<ZE, ZO>(t0, t2);
  a1 = cadd_z<ZE, ZO>(t1, t3);
  a3 = csub_z<ZE, ZO>(t1, t3);
}

// First-stage dft4 of the radix-16 DFT over inputs N2, N2 + 4, N2 + 8, N2 + 12; bit r of LIVE
// clear means that input r is known to be zero.
template <bool INV, unsigned LIVE, int N2>
__device__ __forceinline__ void dft16_stage1(float2* v) {
  dft4_z<INV, !((LIVE >> N2) & 1u), !((LIVE >> (N2 + 4)) & 1u), !((LIVE >> (N2 + 8)) & 1u),
         !((LIVE >> (N2 + 12)) & 1u)>(v[N2], v[N2 + 4], v[N2 + 8], v[N2 + 12]);
}

template <bool INV, unsigned LIVE = 0xFFFFu>
__device__ __forceinline__ void dft16(float2* v) {
  // 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
  dft16_stage1<INV, LIVE, 0>(v);
  dft16_stage1<INV, LIVE, 1>(v);
  dft16_stage1<INV, LIVE, 2>(v);
  dft16_stage1<INV, LIVE, 3>(v);
  // after this, v[n2 + 4 k1] holds Y[n2][k1]; twiddle by w16^(n2 k1)
  v[5] = cmul(v[5], w16<INV>(1));
  v[6] = cmul(v[6], w16<INV>(2));
  v[7] = cmul(v[7], w16<INV>(3));
  v[9] = cmul(v[9], w16<INV>(2));
  v[10] = mul_mi<INV>(v[10]);
  v[11] = cmul(v[11], w16<INV>(6));
  v[13] = cmul(v[13], w16<INV>(3));
  v[14] = cmul(v[14], w16<INV>(6));
  v[15] = cmul(v[15], w16<INV>(9));
  float2 o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a0 = v[4 * k1], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
    dft4<INV>(a0, a1, a2, a3);
    o[k1] = a0;
    o[k1 + 4] = a1;
    o[k1 + 8] = a2;
    o[k1 + 12] = a3;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = o[i];
}

template <int R, bool INV>
__device__ __forceinline__ void dft_r(float2* v) {
  if constexpr (R == 2) dft2<INV>(v[0], v[1]);
  else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<INV>(v);
  else dft16<INV>(v);
}

}  // namespace grafx
