// Zero-phase FIR equaliser (paper Sec. 3 "Equalizer", Eqs. 4-5): 2047 taps designed from 1024
// log-magnitudes, applied to both channels.
//
// Design (once per render, all EQ nodes): h[n] = v[n] (A_0 + 2 sum_k A_k cos(2 pi k n / 2047)) /
// 2047 with A_k = exp(p_k) and a symmetric Hann window v, accumulated in double; then the real
// spectrum of h on the 4096-point grid, H[k] = h[0] + 2 sum_n h[n] cos(2 pi k n / 4096), scaled
// by 1/4096 for the inverse transform.
//
// Filtering: overlap-save, one 4096-point complex FFT per tile of 2048 outputs. The two
// channels ride in one complex signal (left + i right); the filter is real and even, so
// multiplying the spectrum by real H filters both channels at once. A tile's window starts 1024
// samples before its first output, so the 2047-tap kernel never wraps. The FFT is a radix-16
// Stockham transform with 256 threads x 16 points held in registers: the forward transform ends
// and the inverse begins in the same register layout, so only the two inner passes of each
// transform touch LDS. Tiles of one node are mapped onto one XCD (neighbouring tiles share the
// halo through its L2).
//
// Adjoint: the input adjoint is the same filter applied to the output adjoint (h is even). The
// FIR gradient hbar[n] = sum_{c,t} ybar_c[t] u_c[t - n] is the real part of a complex
// correlation, accumulated per tile as W'[k] conj(U_tile[k]) (ybar window spectrum times the
// conjugate spectrum of the zero-padded input tile); each block sums the cross-spectra of a
// fixed group of tiles, the groups are summed in a fixed order, one inverse FFT gives hbar, and
// the chain rule through the design gives dL/dp_k = (kappa_k / 2047) A_k sum_n hbar[n] v[n]
// cos(2 pi k n / 2047).
#include "device_common.h"
#include "grafx_internal.h"
#include "kernels.h"
#include "tables.inc"

namespace grafx {
namespace {

constexpr int kN = kEqFFT;
constexpr int kLds = kN + kN / 16;  // one pad slot per 16 entries

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

template <bool INV>
__device__ __forceinline__ float2 twiddle(int m) {
  const float2 w = kTw4096[m];
  return INV ? make_float2(w.x, -w.y) : w;
}

// In-place 4096-point DFT (forward: exp(-2 pi i nk/N); inverse: exp(+...), unnormalised).
// On entry v[r] holds x[j + 256 r] for thread j; on exit v[r] holds X[j + 256 r].
template <bool INV>
__device__ __forceinline__ void fft4096(float2 (&v)[16], float2* lds) {
  const int j = threadIdx.x;
  // pass 0 (sub-transform size 1): no twiddles
  dft16<INV>(v);
#pragma unroll
  for (int r = 0; r < 16; ++r) lds[pad(16 * j + r)] = v[r];
  __syncthreads();
  // pass 1 (sub-transform size 16)
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = lds[pad(j + 256 * r)];
  {
    const int k = j & 15;
#pragma unroll
    for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twiddle<INV>(r * k * 16));
  }
  dft16<INV>(v);
  __syncthreads();
  {
    const int base = (j >> 4) * 256 + (j & 15);
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[pad(base + 16 * r)] = v[r];
  }
  __syncthreads();
  // pass 2 (sub-transform size 256): outputs land at j + 256 r
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = lds[pad(j + 256 * r)];
#pragma unroll
  for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twiddle<INV>(r * j));
  dft16<INV>(v);
  __syncthreads();
}

// ---- design ---------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void eq_design_h_kernel(const float* P, double* h) {
  __shared__ double A[1024];
  __shared__ double cs[2047];
  const int slot = blockIdx.x;
  for (int i = threadIdx.x; i < 1024; i += kBlock) A[i] = exp((double)P[(int64_t)slot * 1024 + i]);
  for (int i = threadIdx.x; i < 2047; i += kBlock) cs[i] = kCos2047[i];
  __syncthreads();
  const int n = blockIdx.y * kBlock + threadIdx.x;  // 0..1023
  double acc = 0.0;
  int m = 0;
  for (int k = 1; k < 1024; ++k) {
    m += n;
    if (m >= 2047) m -= 2047;
    acc += A[k] * cs[m];
  }
  const double h0 = (A[0] + 2.0 * acc) / 2047.0;
  const double win = 0.5 + 0.5 * cospi((double)n / 1023.0);
  h[(int64_t)slot * 1024 + n] = win * h0;
}

__global__ __launch_bounds__(kBlock) void eq_design_H_kernel(const double* h, float* H) {
  __shared__ double hs[1024];
  __shared__ double cs[kN];
  const int slot = blockIdx.x;
  for (int i = threadIdx.x; i < 1024; i += kBlock) hs[i] = h[(int64_t)slot * 1024 + i];
  for (int i = threadIdx.x; i < kN; i += kBlock) cs[i] = kCos4096[i];
  __syncthreads();
  const int k = blockIdx.y * kBlock + threadIdx.x;
  if (k > kN / 2) return;
  double acc = 0.0;
  int m = 0;
  for (int n = 1; n < 1024; ++n) {
    m = (m + k) & (kN - 1);
    acc += hs[n] * cs[m];
  }
  const float Hk = (float)((hs[0] + 2.0 * acc) / (double)kN);
  float* Hn = H + (int64_t)slot * kN;
  Hn[k] = Hk;
  if (k > 0 && k < kN / 2) Hn[kN - k] = Hk;
}

// ---- forward ----------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void eq_fwd_kernel(GraphView g, float* U, const float* H,
                                                        int node_begin, int tiles) {
  __shared__ float2 lds[kLds];
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int tile = lb % tiles, node = node_begin + lb / tiles;
  const int j = threadIdx.x;
  const int64_t T = g.T;
  const int64_t t0 = (int64_t)tile * kEqHop;
  const int64_t w0 = t0 - kN / 4;  // window start: 1024 samples of history
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = make_float2(0.f, 0.f);
  const int e0 = g.in_ptr[node], e1 = g.in_ptr[node + 1];
  for (int e = e0; e < e1; ++e) {
    const float* row = out_row(g, g.in_src[e]);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t t = w0 + j + 256 * r;
      if (t >= 0 && t < T) {
        v[r].x += row[t];
        v[r].y += row[T + t];
      }
    }
  }
  fft4096<false>(v, lds);
  const float* Hn = H + (int64_t)g.param_row[node] * kN;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const float hk = Hn[j + 256 * r];
    v[r].x *= hk;
    v[r].y *= hk;
  }
  fft4096<true>(v, lds);
  float* y = U + (int64_t)node * 2 * T;
#pragma unroll
  for (int r = 4; r < 12; ++r) {
    const int64_t t = t0 + j + 256 * (r - 4);
    if (t < T) {
      y[t] = v[r].x;
      y[T + t] = v[r].y;
    }
  }
}

// ---- adjoint ----------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void eq_bwd_kernel(GraphView g, float* dU, const float* H,
                                                        int node_begin, int tiles, int groups,
                                                        int tiles_per_group, float2* Cpart) {
  __shared__ float2 lds[kLds];
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int group = lb % groups, node = node_begin + lb / groups;
  const int j = threadIdx.x;
  const int64_t T = g.T;
  const int slot = g.param_row[node];
  const float* Hn = H + (int64_t)slot * kN;
  float* d = dU + (int64_t)node * 2 * T;
  const int o0 = g.out_ptr[node], o1 = g.out_ptr[node + 1];
  const int i0 = g.in_ptr[node], i1 = g.in_ptr[node + 1];
  float2 C[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) C[r] = make_float2(0.f, 0.f);
  const int tile_end = min(tiles, (group + 1) * tiles_per_group);
  for (int tile = group * tiles_per_group; tile < tile_end; ++tile) {
    const int64_t t0 = (int64_t)tile * kEqHop;
    const int64_t w0 = t0 - kN / 4;
    float2 v[16], c[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = make_float2(0.f, 0.f);
    for (int e = o0; e < o1; ++e) {  // output adjoint over the window
      const float* row = adj_row(g, g.out_dst[e]);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t t = w0 + j + 256 * r;
        if (t >= 0 && t < T) {
          v[r].x += row[t];
          v[r].y += row[T + t];
        }
      }
    }
    fft4096<false>(v, lds);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      c[r] = v[r];
      const float hk = Hn[j + 256 * r];
      v[r].x *= hk;
      v[r].y *= hk;
    }
    fft4096<true>(v, lds);
#pragma unroll
    for (int r = 4; r < 12; ++r) {
      const int64_t t = t0 + j + 256 * (r - 4);
      if (t < T) {
        d[t] = v[r].x;
        d[T + t] = v[r].y;
      }
    }
    // input tile, zero-padded to the window (positions 1024..3071)
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = make_float2(0.f, 0.f);
    for (int e = i0; e < i1; ++e) {
      const float* row = out_row(g, g.in_src[e]);
#pragma unroll
      for (int r = 4; r < 12; ++r) {
        const int64_t t = t0 + j + 256 * (r - 4);
        if (t < T) {
          v[r].x += row[t];
          v[r].y += row[T + t];
        }
      }
    }
    fft4096<false>(v, lds);
#pragma unroll
    for (int r = 0; r < 16; ++r) C[r] = cadd(C[r], cmulc(c[r], v[r]));
  }
  float2* out = Cpart + ((int64_t)slot * groups + group) * kN;
#pragma unroll
  for (int r = 0; r < 16; ++r) out[j + 256 * r] = C[r];
}

// Sum the groups' cross-spectra (fixed order), inverse FFT, fold +-n with the window:
// s[0] = hbar[0], s[n] = v[n] (hbar[n] + hbar[-n]).
__global__ __launch_bounds__(kBlock) void eq_grad_reduce_kernel(const float2* Cpart, int groups,
                                                                double* sbuf) {
  __shared__ float2 lds[kLds];
  __shared__ float hb[kN];
  const int slot = blockIdx.x;
  const int j = threadIdx.x;
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    double sx = 0.0, sy = 0.0;
    const float2* p = Cpart + (int64_t)slot * groups * kN + j + 256 * r;
    for (int gi = 0; gi < groups; ++gi) {
      const float2 c = p[(int64_t)gi * kN];
      sx += c.x;
      sy += c.y;
    }
    v[r] = make_float2((float)sx, (float)sy);
  }
  fft4096<true>(v, lds);
#pragma unroll
  for (int r = 0; r < 16; ++r) hb[j + 256 * r] = v[r].x * (1.0f / kN);
  __syncthreads();
  for (int n = j; n < 1024; n += kBlock) {
    double s;
    if (n == 0) {
      s = hb[0];
    } else {
      const double win = 0.5 + 0.5 * cospi((double)n / 1023.0);
      s = win * ((double)hb[n] + (double)hb[kN - n]);
    }
    sbuf[(int64_t)slot * 1024 + n] = s;
  }
}

__global__ __launch_bounds__(kBlock) void eq_grad_p_kernel(const float* P, const double* sbuf,
                                                           float* dP) {
  __shared__ double s[1024];
  __shared__ double cs[2047];
  const int slot = blockIdx.x;
  for (int i = threadIdx.x; i < 1024; i += kBlock) s[i] = sbuf[(int64_t)slot * 1024 + i];
  for (int i = threadIdx.x; i < 2047; i += kBlock) cs[i] = kCos2047[i];
  __syncthreads();
  const int k = blockIdx.y * kBlock + threadIdx.x;  // 0..1023
  double acc = 0.0;
  int m = 0;
  for (int n = 1; n < 1024; ++n) {
    m += k;
    if (m >= 2047) m -= 2047;
    acc += s[n] * cs[m];
  }
  const double A = exp((double)P[(int64_t)slot * 1024 + k]);
  const double kappa = k == 0 ? 1.0 : 2.0;
  dP[(int64_t)slot * 1024 + k] = (float)(kappa / 2047.0 * A * (s[0] + acc));
}

}  // namespace

int eq_tiles(int64_t T) { return (int)((T + kEqHop - 1) / kEqHop); }

static int eq_tiles_per_group(int64_t T) {
  const int tiles = eq_tiles(T);
  int tpg = tiles / 32;
  return tpg < 1 ? 1 : (tpg > 8 ? 8 : tpg);
}

int eq_groups(int64_t T) {
  const int tpg = eq_tiles_per_group(T);
  return (eq_tiles(T) + tpg - 1) / tpg;
}

hipError_t launch_eq_design(const float* P, int n_eq, double* h, float* H, hipStream_t s) {
  if (n_eq <= 0) return hipSuccess;
  eq_design_h_kernel<<<dim3(n_eq, 1024 / kBlock), kBlock, 0, s>>>(P, h);
  eq_design_H_kernel<<<dim3(n_eq, (kN / 2 + kBlock) / kBlock), kBlock, 0, s>>>(h, H);
  return hipGetLastError();
}

hipError_t launch_eq_fwd(const GraphView& g, float* U, const float* H, int node_begin,
                         int n_nodes, hipStream_t s) {
  const int tiles = eq_tiles(g.T);
  eq_fwd_kernel<<<(unsigned)(tiles * n_nodes), kBlock, 0, s>>>(g, U, H, node_begin, tiles);
  return hipGetLastError();
}

hipError_t launch_eq_bwd(const GraphView& g, float* dU, const float* H, int node_begin,
                         int n_nodes, float2* Cpart, hipStream_t s) {
  const int tiles = eq_tiles(g.T), groups = eq_groups(g.T), tpg = eq_tiles_per_group(g.T);
  eq_bwd_kernel<<<(unsigned)(groups * n_nodes), kBlock, 0, s>>>(g, dU, H, node_begin, tiles,
                                                                groups, tpg, Cpart);
  return hipGetLastError();
}

hipError_t launch_eq_grad(const float* P, const float2* Cpart, int n_eq, int groups,
                          double* sbuf, float* dP, hipStream_t s) {
  if (n_eq <= 0) return hipSuccess;
  eq_grad_reduce_kernel<<<n_eq, kBlock, 0, s>>>(Cpart, groups, sbuf);
  eq_grad_p_kernel<<<dim3(n_eq, 1024 / kBlock), kBlock, 0, s>>>(P, sbuf, dP);
  return hipGetLastError();
}

}  // namespace grafx
