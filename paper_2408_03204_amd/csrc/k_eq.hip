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
// transform touch LDS; each thread keeps the 15 twiddles of the last pass in registers for all
// transforms of the block and reads those of the middle pass, which take only 16 x 16 values,
// from LDS. Window gathers use raw buffer loads whose range check supplies the zero padding. Tiles
// of one node are mapped onto one XCD (neighbouring tiles share the halo through its L2); the
// EQ block-order setting can keep the hardware order instead (same arithmetic).
//
// Adjoint: the input adjoint is the same filter applied to the output adjoint (h is even). The
// FIR gradient hbar[n] = sum_{c,t} ybar_c[t] u_c[t - n] is the real part of a complex
// correlation, accumulated per tile as C[k] = W'[k] conj(U_tile[k]) (ybar window spectrum times
// the conjugate spectrum of the zero-padded input tile). The design is even in n, so only
// hbar[n] + hbar[-n] matters: the inverse transform of the real, even sequence
// F[k] = Re C[k] + Re C[N - k], of which N/2 + 1 values are kept. Each block handles one tile
// and writes its folded F into its node's own region; after the last step one launch sums the
// tiles' F per node in a fixed order, which does not depend on how nodes are grouped into steps,
// so results do not depend on the schedule. Then one inverse FFT per node gives
// hbar[n] + hbar[-n], and the chain rule through the design gives
// dL/dp_k = (kappa_k / 2047) A_k sum_n hbar[n] v[n] cos(2 pi k n / 2047).
#include "device_common.h"
#include "grafx_internal.h"
#include "kernels.h"
#include "fft4096.h"
#include "tables.inc"

namespace grafx {
namespace {

using namespace fft4;

// ---- design ----------------------------------------------------------------------------------
// Cosine sums in double, eight lanes per output: lane q sums the terms m = q, q + 8, ... with the
// stride-8 Chebyshev recurrence c_{m+8} = 2 cos(8 theta) c_m - c_{m-8}, so each lane's dependent
// chain is 128 FMAs long; the eight partial sums are combined by a fixed xor butterfly (addition
// is commutative, so all eight lanes end with the same value). Every angle is theta = 2 pi s / M
// for an integer s, so the starting cosines of each lane are read from the table
// tab[i] = cos(2 pi i / M) (correctly rounded) instead of being evaluated.

constexpr int kCosLanes = 8;

template <int M>
__device__ __forceinline__ double cos_sum(const double* w, int s, const double* tab) {
  // sum_{m=1}^{1023} w[m] cos(2 pi m s / M), 0 <= s < 2 M
  const int q = (int)threadIdx.x & (kCosLanes - 1);
  const double two_c8 = 2.0 * tab[(kCosLanes * s) % M];
  double cm = tab[((q - kCosLanes) * s % M + M) % M], c = tab[(q * s) % M];
  double acc = q > 0 ? w[q] * c : 0.0;  // the m = 0 term is not part of the sum
  {
    const double cn = fma(two_c8, c, -cm);
    cm = c;
    c = cn;
  }
#pragma unroll 8
  for (int i = 1; i < 1024 / kCosLanes; ++i) {  // the same trip count on every lane
    acc = fma(w[q + kCosLanes * i], c, acc);
    const double cn = fma(two_c8, c, -cm);
    cm = c;
    c = cn;
  }
#pragma unroll
  for (int d = 1; d < kCosLanes; d <<= 1) acc += __shfl_xor(acc, d, 64);
  return acc;
}

// Outputs handled by one block of the design kernels (kCosLanes threads per output).
constexpr int kCosOut = kBlock / kCosLanes;

__global__ __launch_bounds__(kBlock) void eq_design_h_kernel(const float* P, double* h) {
  __shared__ double A[1024];
  const int slot = blockIdx.x;
  for (int i = threadIdx.x; i < 1024; i += kBlock) A[i] = exp((double)P[(int64_t)slot * 1024 + i]);
  __syncthreads();
  const int n = blockIdx.y * kCosOut + (int)threadIdx.x / kCosLanes;  // 0..1023
  const double h0 = (A[0] + 2.0 * cos_sum<2047>(A, n, kCos2047)) / 2047.0;
  const double win = 0.5 + 0.5 * cospi((double)n / 1023.0);
  if ((threadIdx.x & (kCosLanes - 1)) == 0) h[(int64_t)slot * 1024 + n] = win * h0;
}

__global__ __launch_bounds__(kBlock) void eq_design_H_kernel(const double* h, float* H) {
  __shared__ double hs[1024];
  const int slot = blockIdx.x;
  for (int i = threadIdx.x; i < 1024; i += kBlock) hs[i] = h[(int64_t)slot * 1024 + i];
  __syncthreads();
  const int k = blockIdx.y * kCosOut + (int)threadIdx.x / kCosLanes;
  if (k > kN / 2) return;  // whole groups of kCosLanes lanes leave together
  const float Hk = (float)((hs[0] + 2.0 * cos_sum<kN>(hs, k, kCos4096)) / (double)kN);
  if ((threadIdx.x & (kCosLanes - 1)) != 0) return;
  float* Hn = H + (int64_t)slot * kN;
  Hn[k] = Hk;
  if (k > 0 && k < kN / 2) Hn[kN - k] = Hk;
}

// ---- forward ----------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void eq_fwd_kernel(GraphView g, float* U, const float* H,
                                                        int node_begin, int tiles) {
  __shared__ float2 lds[kLds];
  __shared__ float2 w1lds[kW1Lds];
  const int lb = g.eq_order ? (int)blockIdx.x : xcd_logical_block(blockIdx.x, gridDim.x);
  const int tile = lb % tiles, node = node_begin + lb / tiles;
  const int j = threadIdx.x;
  const int64_t T = g.T, Tn = node_len(g, node);
  const int t0 = tile * kEqHop;
  if (t0 >= Tn) return;  // tile past the node's length
  Twiddles tw;
  load_twiddles(tw, w1lds);
  float2 v[16];
  gather_window<false>(g, node, t0 - kN / 4, v, 0, 16);  // window: 1024 samples of history
  fft4096<false>(v, lds, tw);
  const float* Hn = H + (int64_t)g.param_row[node] * kN;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const float hk = Hn[j + 256 * r];
    v[r].x *= hk;
    v[r].y *= hk;
  }
  fft4096<true>(v, lds, tw);
  float* y = U + (int64_t)node * 2 * T;
  const auto yl = row_rsrc(y, Tn), yr = row_rsrc(y + T, Tn);  // stores past Tn are dropped
#pragma unroll
  for (int r = 4; r < 12; ++r) {
    const int t = t0 + j + 256 * (r - 4);
    bstore_nt(yl, t, v[r].x);
    bstore_nt(yr, t, v[r].y);
  }
}

// ---- adjoint ----------------------------------------------------------------------------------
// Per tile: FFT of the output-adjoint window (its spectrum kept in registers), times H and
// inverse FFT for the input adjoint, FFT of the zero-padded input tile, real part of the
// cross-spectrum through LDS, folded and written per tile.
__global__ __launch_bounds__(kBlock) void eq_bwd_kernel(GraphView g, float* dU, const float* H,
                                                        int node_begin, int tiles, float* Fpart) {
  __shared__ float2 lds[kLds];
  __shared__ float2 w1lds[kW1Lds];
  const int lb = g.eq_order ? (int)blockIdx.x : xcd_logical_block(blockIdx.x, gridDim.x);
  const int tile = lb % tiles, node = node_begin + lb / tiles;
  const int j = threadIdx.x;
  const int64_t T = g.T, Tn = node_len(g, node);
  const int slot = g.param_row[node];
  const float* Hn = H + (int64_t)slot * kN;
  float* d = dU + (int64_t)node * 2 * T;
  float* out = Fpart + ((int64_t)slot * tiles + tile) * kEqFoldStride;
  const int t0 = tile * kEqHop;
  if (t0 >= Tn) {  // tile past the node's length: contributes nothing to the gradient
    for (int k = j; k <= kN / 2; k += kBlock) out[k] = 0.f;
    return;
  }
  Twiddles tw;
  load_twiddles(tw, w1lds);
  float2 v[16], keep[16];
  gather_window<true>(g, node, t0 - kN / 4, v, 0, 16);
  fft4096<false>(v, lds, tw);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    keep[r] = v[r];
    const float hk = Hn[j + 256 * r];
    v[r].x *= hk;
    v[r].y *= hk;
  }
  fft4096<true>(v, lds, tw);
  {
    const auto dl = row_rsrc(d, Tn), dr = row_rsrc(d + T, Tn);  // stores past Tn are dropped
#pragma unroll
    for (int r = 4; r < 12; ++r) {
      const int t = t0 + j + 256 * (r - 4);
      bstore_nt(dl, t, v[r].x);
      bstore_nt(dr, t, v[r].y);
    }
  }
  gather_window<false>(g, node, t0 - kN / 4, v, 4, 12);  // input tile, zero-padded
  fft4096<false, 0x0FF0u>(v, lds, tw);
  // Re C[k] = Re(W'[k] conj(U[k])); fold F[k] = Re C[k] + Re C[N - k], k = 0..N/2 (bins of other
  // threads: through the transform's LDS, free again after its last barrier)
  float* cre = reinterpret_cast<float*>(lds);
#pragma unroll
  for (int r = 0; r < 16; ++r) cre[j + 256 * r] = keep[r].x * v[r].x + keep[r].y * v[r].y;
  __syncthreads();
  for (int k = j; k <= kN / 2; k += kBlock) out[k] = cre[k] + cre[(kN - k) & (kN - 1)];
}

// Sum the folded cross-spectra of the tiles of every EQ node per bin, in double and in a fixed
// order: wave w of a block sums tiles w, w + 4, w + 8, ... of 64 bins, then the four wave sums
// are added in order. Each node has its own region of partials, so one launch after the last
// adjoint step serves every step, and the order does not depend on how nodes form steps.
__global__ __launch_bounds__(kBlock) void eq_fold_reduce_kernel(const float* Fpart, int tiles,
                                                                float* F) {
  __shared__ double part[4][64];
  const int slot = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int k = blockIdx.y * 64 + lane;
  const bool live = k <= kN / 2;
  double s = 0.0;
  if (live) {
    const float* p = Fpart + (int64_t)slot * tiles * kEqFoldStride + k;
#pragma unroll 8
    for (int t = w; t < tiles; t += 4) s += p[(int64_t)t * kEqFoldStride];
  }
  part[w][lane] = s;
  __syncthreads();
  if (w == 0 && live)
    F[(int64_t)slot * kEqFoldStride + k] =
        (float)(((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane]);
}

// The inverse FFT of the folded cross-spectrum gives hbar[n] + hbar[-n]; with the window,
// s[0] = hbar[0] and s[n] = v[n] (hbar[n] + hbar[-n]).
__global__ __launch_bounds__(kBlock) void eq_grad_ifft_kernel(const float* F, double* sbuf) {
  __shared__ float2 lds[kLds];
  __shared__ float hb[kN];
  __shared__ float2 w1lds[kW1Lds];
  const int slot = blockIdx.x;
  const int j = threadIdx.x;
  Twiddles tw;
  load_twiddles(tw, w1lds);
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int k = j + 256 * r;
    v[r] = make_float2(F[(int64_t)slot * kEqFoldStride + (k <= kN / 2 ? k : kN - k)], 0.f);
  }
  fft4096<true>(v, lds, tw);
#pragma unroll
  for (int r = 0; r < 16; ++r) hb[j + 256 * r] = v[r].x * (1.0f / kN);
  __syncthreads();
  for (int n = j; n < 1024; n += kBlock) {
    double s;
    if (n == 0) {
      s = 0.5 * (double)hb[0];
    } else {
      const double win = 0.5 + 0.5 * cospi((double)n / 1023.0);
      s = win * (double)hb[n];
    }
    sbuf[(int64_t)slot * 1024 + n] = s;
  }
}

// dL/dp_k = (kappa_k / 2047) A_k (s[0] + sum_{n>=1} s[n] cos(2 pi k n / 2047)).
__global__ __launch_bounds__(kBlock) void eq_grad_p_kernel(const float* P, const double* sbuf,
                                                           float* dP) {
  __shared__ double s[1024];
  const int slot = blockIdx.x;
  for (int i = threadIdx.x; i < 1024; i += kBlock) s[i] = sbuf[(int64_t)slot * 1024 + i];
  __syncthreads();
  const int k = blockIdx.y * kCosOut + (int)threadIdx.x / kCosLanes;  // 0..1023
  const double acc = cos_sum<2047>(s, k, kCos2047);
  if ((threadIdx.x & (kCosLanes - 1)) != 0) return;
  const double A = exp((double)P[(int64_t)slot * 1024 + k]);
  const double kappa = k == 0 ? 1.0 : 2.0;
  dP[(int64_t)slot * 1024 + k] = (float)(kappa / 2047.0 * A * (s[0] + acc));
}

}  // namespace

int eq_tiles(int64_t T) { return (int)((T + kEqHop - 1) / kEqHop); }

hipError_t launch_eq_design(const float* P, int n_eq, double* h, float* H, hipStream_t s) {
  if (n_eq <= 0) return hipSuccess;
  eq_design_h_kernel<<<dim3(n_eq, 1024 / kCosOut), kBlock, 0, s>>>(P, h);
  eq_design_H_kernel<<<dim3(n_eq, (kN / 2 + kCosOut) / kCosOut), kBlock, 0, s>>>(h, H);
  return hipGetLastError();
}

hipError_t launch_eq_fwd(const GraphView& g, float* U, const float* H, int node_begin,
                         int n_nodes, hipStream_t s) {
  const int tiles = eq_tiles(g.T);
  eq_fwd_kernel<<<(unsigned)(tiles * n_nodes), kBlock, 0, s>>>(g, U, H, node_begin, tiles);
  return hipGetLastError();
}

hipError_t launch_eq_bwd(const GraphView& g, float* dU, const float* H, int node_begin,
                         int n_nodes, float* Fpart, hipStream_t s) {
  const int tiles = eq_tiles(g.T);
  eq_bwd_kernel<<<(unsigned)(tiles * n_nodes), kBlock, 0, s>>>(g, dU, H, node_begin, tiles,
                                                               Fpart);
  return hipGetLastError();
}

hipError_t launch_eq_grad(const float* P, const float* Fpart, int tiles, float* F, int n_eq,
                          double* sbuf, float* dP, hipStream_t s) {
  if (n_eq <= 0) return hipSuccess;
  eq_fold_reduce_kernel<<<dim3(n_eq, (kN / 2 + 64) / 64), kBlock, 0, s>>>(Fpart, tiles, F);
  eq_grad_ifft_kernel<<<n_eq, kBlock, 0, s>>>(F, sbuf);
  eq_grad_p_kernel<<<dim3(n_eq, 1024 / kCosOut), kBlock, 0, s>>>(P, sbuf, dP);
  return hipGetLastError();
}

}  // namespace grafx
