// Filtered-noise mid/side reverb (paper Sec. 3 "Reverb", Eqs. 6-7) and its adjoint.
//
// Impulse response (once per render, every reverb node): a fixed noise realisation, one signal
// for mid and one for side, is analysed by an STFT (384-point frames, hop 192, periodic Hann
// window; frame m covers samples [192 m - 192, 192 m + 192), zero outside the noise); its bins are
// scaled by the mask exp(H0[k] + m HD[k]) (Eq. 7, frames counted from 0; the Nyquist bin takes
// bin 191's mask); every frame goes back through a real inverse DFT, and the frames are
// overlap-added without a synthesis window (the periodic Hann window sums to one at half
// overlap). Mid/side become left/right as in the imager: h_l = (h_m + h_s) / 2,
// h_r = (h_m - h_s) / 2. The noise STFT and the inverse DFTs are direct sums in double
// (384-point frames, 193 one-sided bins); a block makes one hop of h from the two frames that
// overlap there, so no two blocks write one sample.
//
// Filtering: y_c[t] = sum_n h_c[n] u_c[t - n], a causal FIR as long as the noise (two seconds in
// the paper), as uniformly partitioned overlap-save. The FIR is cut into partitions of 2048 taps,
// each zero-padded to 4096 and transformed once per render; the input is transformed once per
// block of 2048 outputs (the 4096-sample window that ends with the block); the spectrum of output
// block b is the sum over partitions p of the spectrum of input window b - p times that of
// partition p, and the second half of its inverse transform is the block. Both channels ride in
// one complex transform (left + i right) and are separated into one-sided per-channel spectra
// (bins 0..2048) when stored, so a product bin needs one load per operand and each thread forms
// bins k and 4096 - k of the packed output spectrum from one product.
//
// Adjoint: the input adjoint is the correlation ubar_c[s] = sum_n h_c[n] ybar_c[s + n], the same
// partitioned product with the conjugate partition spectra over forward-looking windows
// [2048 b, 2048 b + 4096), keeping the first half. Only the spectra Y0[b] of single adjoint blocks
// (placed in the second half of a window) are transformed: a window that starts at block b is
// block b shifted by half a window plus block b + 1, so its spectrum is
// Y0[b + 1][k] + (-1)^k Y0[b][k]. The FIR gradient hbar_c[n] = sum_t ybar_c[t] u_c[t - n] is, per
// partition p, the inverse transform of sum_b Y0_c[b][k] conj(X_c[b - p][k]) (X: the forward's
// input-window spectra, kept in the workspace), first half. It goes back through mid/side, the
// overlap-add (each frame reads its own slice of hbar), the inverse DFT and the mask to dH0 and
// dHD, with per-frame partials summed in frame order.
#include "device_common.h"
#include "fft4096.h"
#include "grafx_internal.h"
#include "kernels.h"

namespace grafx {
namespace {

using namespace fft4;

constexpr int kF = kRvFft;      // 384
constexpr int kHop = kRvHop;    // 192
constexpr int kK = kF / 2 + 1;  // 193 one-sided STFT bins
constexpr int kB = kRvBlock;    // 2048
constexpr int kHalfBins = 9;    // bins k = j + 256 r (r < 9, k <= 2048) of thread j

// exp(+2 pi i j / 384) in double, j = 0..383.
__device__ __forceinline__ void fill_tw384(double2* tw) {
  for (int j = threadIdx.x; j < kF; j += blockDim.x) {
    double s, c;
    sincospi(2.0 * j / kF, &s, &c);
    tw[j] = make_double2(c, s);
  }
}

__device__ __forceinline__ double hann384(int q) { return 0.5 - 0.5 * cospi(2.0 * q / kF); }

// The mask of Eq. 7 at one-sided bin k of frame m for mid (x = 0) or side (x = 1).
__device__ __forceinline__ double mask_at(const float* p, int x, int k, int m) {
  const int kp = k < kRvBins ? k : kRvBins - 1;  // the Nyquist bin shares bin 191's mask
  return exp((double)p[x * 2 * kRvBins + kp] +
             (double)m * (double)p[x * 2 * kRvBins + kRvBins + kp]);
}

// After a forward transform of a packed window (left + i right) held as v[r] = W[j + 256 r]:
// store the one-sided per-channel spectra (L[k], R[k]), k = 0..2048, scaled by `scale`, as
// float4 (L re, L im, R re, R im): L = (W[k] + conj W[N - k]) / 2, R = (W[k] - conj W[N - k]) / 2i.
__device__ __forceinline__ void store_separated(const float2 (&v)[16], float2* lds, float4* out,
                                                float scale) {
  const int j = threadIdx.x;
#pragma unroll
  for (int r = 0; r < 16; ++r) lds[pad(j + 256 * r)] = v[r];
  __syncthreads();
  const float h = 0.5f * scale;
#pragma unroll
  for (int r = 0; r < kHalfBins; ++r) {
    const int k = j + 256 * r;
    if (k > kN / 2) break;
    const float2 w = lds[pad(k)], m = lds[pad((kN - k) & (kN - 1))];
    out[k] = make_float4(h * (w.x + m.x), h * (w.y - m.y), h * (w.y + m.y), h * (m.x - w.x));
  }
}

// Inverse of store_separated for a product held per channel at the thread's one-sided bins:
// writes the packed spectrum Y[k] = L[k] + i R[k] and Y[N - k] = conj L[k] + i conj R[k] into
// LDS and reads it back in the transform's layout (v[r] = Y[j + 256 r]).
__device__ __forceinline__ void pack_spectrum(const float2 (&al)[kHalfBins],
                                              const float2 (&ar)[kHalfBins], float2* lds,
                                              float2 (&v)[16]) {
  const int j = threadIdx.x;
#pragma unroll
  for (int r = 0; r < kHalfBins; ++r) {
    const int k = j + 256 * r;
    if (k > kN / 2) break;
    lds[pad(k)] = make_float2(al[r].x - ar[r].y, al[r].y + ar[r].x);
    if (k != 0 && k != kN / 2)
      lds[pad(kN - k)] = make_float2(al[r].x + ar[r].y, ar[r].x - al[r].y);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = lds[pad(j + 256 * r)];
  __syncthreads();  // the transform overwrites the LDS
}

// ---- noise STFT -------------------------------------------------------------------------------
// Un[x][m][k] = sum_q w[q] noise_x[192 m - 192 + q] e^(-2 pi i k q / 384), k = 0..192.
__global__ __launch_bounds__(kBlock) void rv_noise_stft_kernel(const float* noise, int64_t L,
                                                               int M, double2* Un) {
  __shared__ double fr[kF];
  __shared__ double2 tw[kF];
  const int m = blockIdx.x, x = blockIdx.y;
  fill_tw384(tw);
  for (int q = threadIdx.x; q < kF; q += kBlock) {
    const int64_t n = (int64_t)kHop * m - kHop + q;
    fr[q] = (n >= 0 && n < L) ? hann384(q) * (double)noise[x * L + n] : 0.0;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kK; k += kBlock) {
    double re = 0.0, im = 0.0;
    for (int q = 0; q < kF; ++q) {
      const double2 w = tw[(k * q) % kF];  // e^(+i theta); the analysis takes e^(-i theta)
      re = fma(fr[q], w.x, re);
      im = fma(-fr[q], w.y, im);
    }
    Un[((int64_t)x * M + m) * kK + k] = make_double2(re, im);
  }
}

// ---- impulse response -------------------------------------------------------------------------
// Block (hop s, reverb slot), thread t: sample n = 192 s + t of h_m and h_s, from the second half
// of frame s and the first half of frame s + 1, then left/right.
__global__ __launch_bounds__(kHop) void rv_ir_kernel(const float* P, const double2* Un, int64_t L,
                                                     int M, float* h) {
  __shared__ double2 tw[kF];
  __shared__ double2 X[2][2][kK];  // [mid, side][frame s, s + 1][bin]
  const int s = blockIdx.x, slot = blockIdx.y;
  const float* p = P + (int64_t)slot * kRvParams;
  fill_tw384(tw);
  for (int i = threadIdx.x; i < 2 * 2 * kK; i += kHop) {
    const int x = i / (2 * kK), f = (i / kK) % 2, k = i % kK;
    const int m = s + f;
    const double mu = mask_at(p, x, k, m);
    const double2 u = Un[((int64_t)x * M + m) * kK + k];
    X[x][f][k] = make_double2(u.x * mu, u.y * mu);
  }
  __syncthreads();
  const int t = threadIdx.x;
  double hx[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    double acc = 0.0;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      // real inverse DFT at q: (X[0] + (-1)^q X[192] + 2 sum_{k=1}^{191} Re(X[k] e^(i theta))) / N
      const int q = f == 0 ? kHop + t : t;
      const double2* Xf = X[x][f];
      const double a = Xf[0].x + ((q & 1) ? -Xf[kK - 1].x : Xf[kK - 1].x);
      double b = 0.0;
      for (int k = 1; k < kK - 1; ++k) {
        const double2 w = tw[(k * q) % kF];
        b = fma(Xf[k].x, w.x, b);
        b = fma(-Xf[k].y, w.y, b);
      }
      acc += (a + 2.0 * b) / kF;
    }
    hx[x] = acc;
  }
  const int64_t n = (int64_t)kHop * s + t;
  if (n < L) {
    float* hs = h + (int64_t)slot * 2 * L;
    hs[n] = (float)(0.5 * (hx[0] + hx[1]));
    hs[L + n] = (float)(0.5 * (hx[0] - hx[1]));
  }
}

// ---- partition spectra ------------------------------------------------------------------------
// Partition p of the stereo FIR (taps 2048 p .. 2048 p + 2047, zero-padded to 4096), scaled by
// 1 / 4096 for the unnormalised inverse transforms of the products.
__global__ __launch_bounds__(kBlock) void rv_partition_kernel(const float* h, int64_t L, int parts,
                                                              float4* Hs) {
  __shared__ float2 lds[kLds];
  __shared__ float2 w1lds[kW1Lds];
  const int p = blockIdx.x, slot = blockIdx.y;
  const int j = threadIdx.x;
  Twiddles tw;
  load_twiddles(tw, w1lds);
  const float* hl = h + (int64_t)slot * 2 * L;
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t n = (int64_t)kB * p + j + 256 * r;
    v[r] = (r < 8 && n < L) ? make_float2(hl[n], hl[L + n]) : make_float2(0.f, 0.f);
  }
  fft4096<false>(v, lds, tw);
  store_separated(v, lds, Hs + ((int64_t)slot * parts + p) * kRvStride, 1.0f / kN);
}

// ---- block spectra ----------------------------------------------------------------------------
// ADJ false: input window [2048 b - 2048 + shift, 2048 b + 2048 + shift) of the node's input sum;
// ADJ true: output-adjoint block [2048 b + shift, 2048 b + 2048 + shift) in the second half of a
// zero window. Stored at the node's parameter slot.
template <bool ADJ>
__global__ __launch_bounds__(kBlock) void rv_spectra_kernel(GraphView g, int node_begin, int nb,
                                                            int shift, float4* out) {
  __shared__ float2 lds[kLds];
  __shared__ float2 w1lds[kW1Lds];
  const int b = blockIdx.x, node = node_begin + blockIdx.y;
  const int slot = g.param_row[node];
  Twiddles tw;
  load_twiddles(tw, w1lds);
  float2 v[16];
  gather_window<ADJ>(g, node, kB * b - kB + shift, v, ADJ ? 8 : 0, 16);
  fft4096<false>(v, lds, tw);
  store_separated(v, lds, out + ((int64_t)slot * nb + b) * kRvStride, 1.0f);
}

// ---- partitioned product and inverse ------------------------------------------------------------
// Forward (CORR false): output block b = second half of IFFT(sum_{p <= b} X[b - p] H[p]).
// Adjoint (CORR true): input-adjoint block b = first half of IFFT(sum_p Yf[b + p] conj(H[p])) with
// Yf[c] = Y0[c + 1] + (-1)^k Y0[c] (zero past the last block).
template <bool CORR>
__global__ __launch_bounds__(kBlock) void rv_product_kernel(GraphView g, float* out, int node_begin,
                                                            int nb, int parts, const float4* S,
                                                            const float4* Hs) {
  __shared__ float2 lds[kLds];
  __shared__ float2 w1lds[kW1Lds];
  const int b = blockIdx.x, node = node_begin + blockIdx.y;
  const int slot = g.param_row[node];
  const int j = threadIdx.x;
  const int64_t T = g.T, Tn = node_len(g, node);
  if ((int64_t)kB * b >= Tn) return;  // block past the node's length (uniform over the block)
  Twiddles tw;
  load_twiddles(tw, w1lds);
  const float4* Ss = S + (int64_t)slot * nb * kRvStride;
  const float4* Hn = Hs + (int64_t)slot * parts * kRvStride;
  const float sgn = (j & 1) ? -1.f : 1.f;  // (-1)^k for every bin k = j + 256 r of this thread
  float2 al[kHalfBins], ar[kHalfBins];
#pragma unroll
  for (int r = 0; r < kHalfBins; ++r) al[r] = ar[r] = make_float2(0.f, 0.f);
  const int np = CORR ? min(parts, nb - b) : min(parts, b + 1);
  for (int p = 0; p < np; ++p) {
    const float4* hp = Hn + (int64_t)p * kRvStride;
    const float4* z0 = Ss + (int64_t)(CORR ? b + p : b - p) * kRvStride;
    const bool has_next = CORR && b + p + 1 < nb;
#pragma unroll
    for (int r = 0; r < kHalfBins; ++r) {
      const int k = j + 256 * r;
      if (k > kN / 2) break;
      float4 z = z0[k];
      if (CORR) {
        z = make_float4(sgn * z.x, sgn * z.y, sgn * z.z, sgn * z.w);
        if (has_next) {
          const float4 z1 = z0[kRvStride + k];
          z = make_float4(z.x + z1.x, z.y + z1.y, z.z + z1.z, z.w + z1.w);
        }
      }
      const float4 hh = hp[k];
      const float2 hl = CORR ? make_float2(hh.x, -hh.y) : make_float2(hh.x, hh.y);
      const float2 hr = CORR ? make_float2(hh.z, -hh.w) : make_float2(hh.z, hh.w);
      al[r] = cadd(al[r], cmul(make_float2(z.x, z.y), hl));
      ar[r] = cadd(ar[r], cmul(make_float2(z.z, z.w), hr));
    }
  }
  float2 v[16];
  pack_spectrum(al, ar, lds, v);
  fft4096<true>(v, lds, tw);
  float* y = out + (int64_t)node * 2 * T;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int64_t t = (int64_t)kB * b + j + 256 * r;
    if (t < Tn) {
      const float2 o = v[CORR ? r : r + 8];
      y[t] = o.x;
      y[T + t] = o.y;
    }
  }
}

// ---- FIR gradient (the partitioned cross-correlation) ---------------------------------------------
// Cross-spectrum of partition p per channel, one-sided bins: G_c[k] = sum_{b >= p} Y0_c[b][k]
// conj(X_c[b - p][k]), summed in block order in double, scaled by 1 / 4096.
__global__ __launch_bounds__(kBlock) void rv_cross_kernel(int nb, int parts, const float4* Y0,
                                                          const float4* X, float4* Gs) {
  const int p = blockIdx.x, k = blockIdx.y * kBlock + threadIdx.x;
  const int slot = blockIdx.z;
  if (k > kN / 2) return;
  const float4* ys = Y0 + (int64_t)slot * nb * kRvStride + k;
  const float4* xs = X + (int64_t)slot * nb * kRvStride + k;
  double lre = 0.0, lim = 0.0, rre = 0.0, rim = 0.0;
  for (int b = p; b < nb; ++b) {
    const float4 y = ys[(int64_t)b * kRvStride], x = xs[(int64_t)(b - p) * kRvStride];
    lre += (double)y.x * x.x + (double)y.y * x.y;
    lim += (double)y.y * x.x - (double)y.x * x.y;
    rre += (double)y.z * x.z + (double)y.w * x.w;
    rim += (double)y.w * x.z - (double)y.z * x.w;
  }
  constexpr double s = 1.0 / kN;
  Gs[((int64_t)slot * parts + p) * kRvStride + k] =
      make_float4((float)(s * lre), (float)(s * lim), (float)(s * rre), (float)(s * rim));
}

// hbar_c[2048 p + i] = first half of the inverse transform of G (left: real part, right:
// imaginary part of the packed transform G_l + i G_r).
__global__ __launch_bounds__(kBlock) void rv_hbar_kernel(const float4* Gs, int parts, int64_t L,
                                                         float* hbar) {
  __shared__ float2 lds[kLds];
  __shared__ float2 w1lds[kW1Lds];
  const int p = blockIdx.x, slot = blockIdx.y;
  const int j = threadIdx.x;
  Twiddles tw;
  load_twiddles(tw, w1lds);
  const float4* G = Gs + ((int64_t)slot * parts + p) * kRvStride;
  float2 al[kHalfBins], ar[kHalfBins];
#pragma unroll
  for (int r = 0; r < kHalfBins; ++r) {
    const int k = j + 256 * r;
    const float4 q = k <= kN / 2 ? G[k] : make_float4(0.f, 0.f, 0.f, 0.f);
    al[r] = make_float2(q.x, q.y);
    ar[r] = make_float2(q.z, q.w);
  }
  float2 v[16];
  pack_spectrum(al, ar, lds, v);
  fft4096<true>(v, lds, tw);
  float* hb = hbar + (int64_t)slot * 2 * L;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int64_t n = (int64_t)kB * p + j + 256 * r;
    if (n < L) {
      hb[n] = v[r].x;
      hb[L + n] = v[r].y;
    }
  }
}

// Per frame m and mid/side x: fbar[q] = hbar_x[192 m - 192 + q] (hbar_m = (hbar_l + hbar_r) / 2,
// hbar_s = (hbar_l - hbar_r) / 2), V[k] = sum_q fbar[q] e^(2 pi i k q / 384), and the gradient with
// respect to the log-mask entry (k, m): (c_k / 384) Re(Un[k] V[k]) mu[k] (c_k = 1 at k = 0 and
// 192, else 2).
__global__ __launch_bounds__(kBlock) void rv_frame_grad_kernel(const float* P, const double2* Un,
                                                               const float* hbar, int64_t L, int M,
                                                               double* part) {
  __shared__ double2 tw[kF];
  __shared__ double fb[kF];
  const int m = blockIdx.x, x = blockIdx.y, slot = blockIdx.z;
  fill_tw384(tw);
  const float* hb = hbar + (int64_t)slot * 2 * L;
  for (int q = threadIdx.x; q < kF; q += kBlock) {
    const int64_t n = (int64_t)kHop * m - kHop + q;
    double v = 0.0;
    if (n >= 0 && n < L) v = 0.5 * ((double)hb[n] + (x == 0 ? 1.0 : -1.0) * (double)hb[L + n]);
    fb[q] = v;
  }
  __syncthreads();
  const float* p = P + (int64_t)slot * kRvParams;
  for (int k = threadIdx.x; k < kK; k += kBlock) {
    double re = 0.0, im = 0.0;
    for (int q = 0; q < kF; ++q) {
      const double2 w = tw[(k * q) % kF];
      re = fma(fb[q], w.x, re);
      im = fma(fb[q], w.y, im);
    }
    const double2 u = Un[((int64_t)x * M + m) * kK + k];
    const double c = (k == 0 || k == kK - 1) ? 1.0 : 2.0;
    part[(((int64_t)slot * 2 + x) * M + m) * kK + k] =
        c / kF * (u.x * re - u.y * im) * mask_at(p, x, k, m);
  }
}

// dH0[k] = sum_m G[m][k], dHD[k] = sum_m m G[m][k], in frame order (bin 191 adds the Nyquist
// bin, which shares its mask).
__global__ __launch_bounds__(kBlock) void rv_param_grad_kernel(const double* part, int M,
                                                               float* dP) {
  const int slot = blockIdx.x, x = blockIdx.y, k = threadIdx.x;
  if (k >= kRvBins) return;
  const double* ps = part + ((int64_t)slot * 2 + x) * M * kK;
  double a = 0.0, d = 0.0;
  for (int m = 0; m < M; ++m) {
    double gm = ps[(int64_t)m * kK + k];
    if (k == kRvBins - 1) gm += ps[(int64_t)m * kK + kK - 1];
    a += gm;
    d = fma((double)m, gm, d);
  }
  float* out = dP + (int64_t)slot * kRvParams + x * 2 * kRvBins;
  out[k] = (float)a;
  out[kRvBins + k] = (float)d;
}

}  // namespace

int rv_frames(int64_t L) { return (int)((L + kHop - 1) / kHop) + 1; }
int rv_parts(int64_t L) { return (int)((L + kB - 1) / kB); }
int rv_blocks(int64_t T) { return (int)((T + kB - 1) / kB); }

hipError_t launch_rv_design(const float* P, int n, const float* noise, int64_t L, double2* Un,
                            float* h, float4* Hs, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int M = rv_frames(L), parts = rv_parts(L);
  rv_noise_stft_kernel<<<dim3(M, 2), kBlock, 0, s>>>(noise, L, M, Un);
  rv_ir_kernel<<<dim3(M - 1, n), kHop, 0, s>>>(P, Un, L, M, h);
  rv_partition_kernel<<<dim3(parts, n), kBlock, 0, s>>>(h, L, parts, Hs);
  return hipGetLastError();
}

hipError_t launch_xcorr_spectra(const GraphView& g, int node_begin, int n_nodes, bool adj,
                                int shift, int nb, float4* out, hipStream_t s) {
  if (adj)
    rv_spectra_kernel<true><<<dim3(nb, n_nodes), kBlock, 0, s>>>(g, node_begin, nb, shift, out);
  else
    rv_spectra_kernel<false><<<dim3(nb, n_nodes), kBlock, 0, s>>>(g, node_begin, nb, shift, out);
  return hipGetLastError();
}

hipError_t launch_xcorr(int n, int nb, int parts, int64_t len, const float4* Y0, const float4* X,
                        float4* Gs, float* R, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  rv_cross_kernel<<<dim3(parts, (kN / 2 + kBlock) / kBlock, n), kBlock, 0, s>>>(nb, parts, Y0, X,
                                                                                 Gs);
  rv_hbar_kernel<<<dim3(parts, n), kBlock, 0, s>>>(Gs, parts, len, R);
  return hipGetLastError();
}

hipError_t launch_rv_fwd(const GraphView& g, float* U, int node_begin, int n_nodes, int64_t L,
                         const float4* Hs, float4* Z, hipStream_t s) {
  const int nb = rv_blocks(g.T), parts = rv_parts(L);
  rv_spectra_kernel<false><<<dim3(nb, n_nodes), kBlock, 0, s>>>(g, node_begin, nb, 0, Z);
  rv_product_kernel<false><<<dim3(nb, n_nodes), kBlock, 0, s>>>(g, U, node_begin, nb, parts, Z,
                                                                Hs);
  return hipGetLastError();
}

hipError_t launch_rv_bwd(const GraphView& g, float* dU, int node_begin, int n_nodes, int64_t L,
                         const float4* Hs, float4* Y0, hipStream_t s) {
  const int nb = rv_blocks(g.T), parts = rv_parts(L);
  rv_spectra_kernel<true><<<dim3(nb, n_nodes), kBlock, 0, s>>>(g, node_begin, nb, 0, Y0);
  rv_product_kernel<true><<<dim3(nb, n_nodes), kBlock, 0, s>>>(g, dU, node_begin, nb, parts, Y0,
                                                               Hs);
  return hipGetLastError();
}

hipError_t launch_rv_grad(int n, int64_t T, int64_t L, const float* P, const double2* Un,
                          const float4* Z, const float4* Y0, float4* Gs, float* hbar,
                          double* part, float* dP, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nb = rv_blocks(T), parts = rv_parts(L), M = rv_frames(L);
  const hipError_t e = launch_xcorr(n, nb, parts, L, Y0, Z, Gs, hbar, s);
  if (e != hipSuccess) return e;
  rv_frame_grad_kernel<<<dim3(M, 2, n), kBlock, 0, s>>>(P, Un, hbar, L, M, part);
  rv_param_grad_kernel<<<dim3(n, 2), kBlock, 0, s>>>(part, M, dP);
  return hipGetLastError();
}

}  // namespace grafx
