// Filtered-noise mid/side reverb (paper Sec. 3 "Reverb", Eqs. 6-7) and its adjoint.
//
// Impulse response (once per render, every reverb node): a fixed noise realisation, one signal
// for mid and one for side, is analysed by an STFT (384-point frames, hop 192, periodic Hann
// window; frame m covers samples [192 m - 192, 192 m + 192), zero outside the noise); its bins are
// scaled by the mask exp(H0[k] + m HD[k]) (Eq. 7, frames counted from 0; the Nyquist bin takes
// bin 191's mask); every frame goes back through a real inverse DFT, and the frames are
// overlap-added without a synthesis window (the periodic Hann window sums to one at half
// overlap). Mid/side become left/right as in the imager: h_l = (h_m + h_s) / 2,
// h_r = (h_m - h_s) / 2. The noise STFT is a direct sum in double; a hop of h is one real inverse
// DFT (in double) of the two masked frames that overlap there, combined in the frequency domain.
//
// Filtering: y_c[t] = sum_n h_c[n] u_c[t - n], a causal FIR as long as the noise (two seconds in
// the paper), as uniformly partitioned overlap-save. The FIR is cut into partitions of 2048 taps,
// each zero-padded to 4096 and transformed once per render; the input is transformed once per
// block of 2048 outputs (the 4096-sample window that ends with the block); the spectrum of output
// block b is the sum over partitions p of the spectrum of input window b - p times that of
// partition p, and the second half of its inverse transform is the block. Both channels ride in
// one complex transform (left + i right) and are separated into one-sided per-channel spectra
// (bins 0..2048) when stored. The sum over partitions runs bin-major (a thread per bin, the
// partition spectra in registers, the blocks streaming through), its partial spectra per tile of
// partitions go through the workspace, and a second kernel rebuilds each block's packed spectrum
// and transforms it back.
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
// dHD, with partials per group of frames summed in a fixed order.
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
// Sample 192 s + t of h_x (t < 192) is the sum of frame s at q = 192 + t and frame s + 1 at q = t.
// Since e^(2 pi i k (192 + t) / 384) = (-1)^k e^(2 pi i k t / 384), that is one real inverse DFT
// per hop s of the combined spectrum Y_s[k] = c_k / 384 (X_{s+1}[k] + (-1)^k X_s[k]), X_m the
// masked frame spectrum and c_k = 1 at k = 0, 192, else 2: h_x[192 s + t] = sum_k Re(Y_s[k]
// e^(2 pi i k t / 384)). A block takes kIrHops hops of one reverb slot: Y of both channels in LDS
// (double), then each thread sums, for three samples t = r, r + 64, r + 128 and four hops, both
// channels (24 accumulators), stepping the three twiddles by multiplication (restarted from exact
// values every 64 bins); a wave's lanes all read the same Y entry (LDS broadcast).
constexpr int kIrHops = 8;                 // hops per block
constexpr int kIrHopsPerWave = 4;          // hops per wave (two waves)
constexpr int kIrThreads = 128;

__global__ __launch_bounds__(kIrThreads) void rv_ir_kernel(const float* P, const double2* Un,
                                                           int64_t L, int M, float* h) {
  __shared__ double2 Y[2][kIrHops][kK];
  const int s0 = blockIdx.x * kIrHops, slot = blockIdx.y;
  const float* p = P + (int64_t)slot * kRvParams;
  for (int i = threadIdx.x; i < 2 * kIrHops * kK; i += kIrThreads) {
    const int x = i / (kIrHops * kK), j = (i / kK) % kIrHops, k = i % kK;
    const int s = s0 + j;
    double2 y = make_double2(0.0, 0.0);
    if (s < M - 1) {
      const double mu0 = mask_at(p, x, k, s), mu1 = mask_at(p, x, k, s + 1);
      const double2 u0 = Un[((int64_t)x * M + s) * kK + k];
      const double2 u1 = Un[((int64_t)x * M + s + 1) * kK + k];
      const double sg = (k & 1) ? -1.0 : 1.0;
      const double c = (k == 0 || k == kK - 1) ? 1.0 / kF : 2.0 / kF;
      y = make_double2(c * (u1.x * mu1 + sg * u0.x * mu0), c * (u1.y * mu1 + sg * u0.y * mu0));
    }
    Y[x][j][k] = y;
  }
  __syncthreads();
  const int r = threadIdx.x & 63, hg = threadIdx.x >> 6;  // sample group, hop group (= wave)
  double acc[3][kIrHopsPerWave][2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < kIrHopsPerWave; ++j) acc[i][j][0] = acc[i][j][1] = 0.0;
  double sr[3], si[3];  // twiddle steps e^(2 pi i t / 384)
#pragma unroll
  for (int i = 0; i < 3; ++i) sincospi(2.0 * (r + 64 * i) / kF, &si[i], &sr[i]);
  for (int k0 = 0; k0 < kK; k0 += 64) {
    double wr[3], wi[3];  // e^(2 pi i k0 t / 384), exactly
#pragma unroll
    for (int i = 0; i < 3; ++i)
      sincospi(2.0 * (double)((k0 * (r + 64 * i)) % kF) / kF, &wi[i], &wr[i]);
    const int k1 = min(k0 + 64, kK);
    for (int k = k0; k < k1; ++k) {
#pragma unroll
      for (int j = 0; j < kIrHopsPerWave; ++j) {
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const double2 y = Y[x][hg * kIrHopsPerWave + j][k];
#pragma unroll
          for (int i = 0; i < 3; ++i) acc[i][j][x] = fma(y.x, wr[i], fma(-y.y, wi[i], acc[i][j][x]));
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double t = wr[i] * sr[i] - wi[i] * si[i];
        wi[i] = fma(wr[i], si[i], wi[i] * sr[i]);
        wr[i] = t;
      }
    }
  }
  float* hs = h + (int64_t)slot * 2 * L;
#pragma unroll
  for (int j = 0; j < kIrHopsPerWave; ++j) {
    const int s = s0 + hg * kIrHopsPerWave + j;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int64_t n = (int64_t)kHop * s + r + 64 * i;
      if (s < M - 1 && n < L) {
        hs[n] = (float)(0.5 * (acc[i][j][0] + acc[i][j][1]));
        hs[L + n] = (float)(0.5 * (acc[i][j][0] - acc[i][j][1]));
      }
    }
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
  fft4096<false, 0x00FFu>(v, lds, tw);
  store_separated(v, lds, Hs + ((int64_t)slot * parts + p) * kRvStride, 1.0f / kN);
}

// ---- block spectra ----------------------------------------------------------------------------
// ADJ false: input window [2048 b - 2048 + shift, 2048 b + 2048 + shift) of the node's input sum;
// ADJ true: output-adjoint block [2048 b + shift, 2048 b + 2048 + shift) in the second half of a
// zero window. Stored at the node's parameter slot.
template <bool ADJ>
__global__ __launch_bounds__(kBlock) void rv_spectra_kernel(GraphView g, int node_begin, int nb,
                                                            int shift, float4* out,
                                                            int32_t* slot_len) {
  __shared__ float2 lds[kLds];
  __shared__ float2 w1lds[kW1Lds];
  const int b = blockIdx.x, node = node_begin + blockIdx.y;
  const int slot = g.param_row[node];
  Twiddles tw;
  load_twiddles(tw, w1lds);
  float2 v[16];
  if (slot_len && b == 0 && threadIdx.x == 0) slot_len[slot] = (int32_t)node_len(g, node);
  gather_window<ADJ>(g, node, kB * b - kB + shift, v, ADJ ? 8 : 0, 16);
  fft4096<false, ADJ ? 0xFF00u : 0xFFFFu>(v, lds, tw);
  store_separated(v, lds, out + ((int64_t)slot * nb + b) * kRvStride, 1.0f);
}

// ---- partitioned product, bin-major -------------------------------------------------------------
// For one one-sided bin k the partitioned product is a short convolution along the block index:
// forward C[b] = sum_p X[b - p] H[p], adjoint C[b] = sum_p Yf[b + p] conj(H[p]) with
// Yf[c] = Y0[c + 1] + (-1)^k Y0[c] (per channel, complex). A thread owns one bin of one node and
// one tile of kConvTile partitions: the tile's partition spectra stay in registers, and the blocks
// enter a register ring one per step (the loop is unrolled by the tile size, so the ring is
// indexed statically), so every stored spectrum is read once per tile instead of once per
// (block, partition) pair. Each tile writes its partial C to the workspace; the inverse kernel
// adds the tiles in order. One wave per block (bins 0..2048 in 33 waves). The block range is cut
// into segments of kConvSeg steps, one wave each, so that a node's chain of dependent loads is
// short; a segment first re-forms the kConvTile - 1 entries before it (its ring warm-up).
constexpr int kConvTile = 22;
constexpr int kConvSeg = 64;
constexpr int kBinWave = 64;
constexpr int kBinWaves = (kN / 2 + kBinWave) / kBinWave;  // 33

__device__ __forceinline__ float4 cmac2(float4 acc, float4 a, float4 b) {
  // per channel (x, y) and (z, w): acc += a * b (complex)
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
  acc.z = fma(a.z, b.z, fma(-a.w, b.w, acc.z));
  acc.w = fma(a.z, b.w, fma(a.w, b.z, acc.w));
  return acc;
}

template <bool CORR>
__global__ __launch_bounds__(kBinWave) void rv_conv_bins_kernel(GraphView g, int node_begin,
                                                                int nb, int parts, int tiles,
                                                                int nseg, const float4* S,
                                                                const float4* Hs, float4* C) {
  const int k = blockIdx.x * kBinWave + threadIdx.x;
  const int tile = blockIdx.y / nseg, seg = blockIdx.y % nseg, node = node_begin + blockIdx.z;
  if (k > kN / 2) return;  // no barriers in this kernel
  const int slot = g.param_row[node];
  const int p0 = tile * kConvTile;
  const float4* Sk = S + (int64_t)slot * nb * kRvStride + k;
  const float4* Hk = Hs + ((int64_t)slot * parts + p0) * kRvStride + k;
  const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 h[kConvTile], ring[kConvTile];
#pragma unroll
  for (int i = 0; i < kConvTile; ++i) {
    // loads from clamped, valid addresses and a select on the value (a select between a global
    // address and a local zero would turn every load into a flat access)
    float4 v = Hk[(int64_t)max(min(i, parts - 1 - p0), 0) * kRvStride];
    if (CORR) v = make_float4(v.x, -v.y, v.z, -v.w);
    h[i] = p0 + i < parts ? v : zero;
    ring[i] = zero;
  }
  const float sg = (k & 1) ? -1.f : 1.f;
  float4* Ck = C + ((int64_t)slot * tiles + tile) * nb * kRvStride + k;
  // steps [qs, qe) are stored; entries from q_start (a multiple of the tile, at least
  // kConvTile - 1 steps before qs) are formed
  const int qs = seg * kConvSeg, qe = min(nb, qs + kConvSeg);
  const int q_start = max(0, qs - (kConvTile - 1)) / kConvTile * kConvTile;
  float4 y_next = zero;  // adjoint: Y0[c + 1] of the entry c being formed
  if (CORR) {
    const int c1 = nb - q_start + p0;  // c + 1 of the first entry
    const float4 yv = Sk[(int64_t)min(c1, nb - 1) * kRvStride];
    y_next = c1 < nb ? yv : zero;
  }
  for (int q0 = q_start; q0 < qe; q0 += kConvTile) {
#pragma unroll
    for (int j = 0; j < kConvTile; ++j) {
      const int q = q0 + j;
      if (q < qe) {  // uniform over the wave
      // step q: the entry of partition p0 enters ring[j]; partition p0 + i reads the entry that
      // entered i steps earlier, ring[(j - i) mod kConvTile]
      const int b = CORR ? nb - 1 - q : q;
      const int c = CORR ? b + p0 : b - p0;
      float4 e;
      if (CORR) {
        const float4 yv = Sk[(int64_t)min(c, nb - 1) * kRvStride];
        const float4 y = c < nb ? yv : zero;
        e = make_float4(y_next.x + sg * y.x, y_next.y + sg * y.y, y_next.z + sg * y.z,
                        y_next.w + sg * y.w);
        y_next = y;
      } else {
        const float4 xv = Sk[(int64_t)max(c, 0) * kRvStride];
        e = c >= 0 ? xv : zero;
      }
      ring[j] = e;
      if (q >= qs) {
        float4 acc = zero;
#pragma unroll
        for (int i = 0; i < kConvTile; ++i)
          acc = cmac2(acc, ring[(j - i + kConvTile) % kConvTile], h[i]);
        Ck[(int64_t)b * kRvStride] = acc;
      }
      }
    }
  }
}

// Output block b: the tiles' partial spectra added in tile order, the packed spectrum rebuilt
// through LDS, one inverse transform; forward keeps its second half, adjoint its first.
template <bool CORR>
__global__ __launch_bounds__(kBlock) void rv_inverse_kernel(GraphView g, float* out, int node_begin,
                                                            int nb, int tiles, const float4* C) {
  __shared__ float2 lds[kLds];
  __shared__ float2 w1lds[kW1Lds];
  const int b = blockIdx.x, node = node_begin + blockIdx.y;
  const int slot = g.param_row[node];
  const int j = threadIdx.x;
  const int64_t T = g.T, Tn = node_len(g, node);
  if ((int64_t)kB * b >= Tn) return;  // block past the node's length (uniform over the block)
  Twiddles tw;
  load_twiddles(tw, w1lds);
  const float4* Cb = C + ((int64_t)slot * tiles * nb + b) * kRvStride;
  float2 al[kHalfBins], ar[kHalfBins];
#pragma unroll
  for (int r = 0; r < kHalfBins; ++r) {
    const int k = j + 256 * r;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (k <= kN / 2)
      for (int t = 0; t < tiles; ++t) {
        const float4 v = Cb[(int64_t)t * nb * kRvStride + k];
        acc = make_float4(acc.x + v.x, acc.y + v.y, acc.z + v.z, acc.w + v.w);
      }
    al[r] = make_float2(acc.x, acc.y);
    ar[r] = make_float2(acc.z, acc.w);
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
      store_nt(y + t, o.x);
      store_nt(y + T + t, o.y);
    }
  }
}

// ---- FIR gradient (the partitioned cross-correlation), bin-major ---------------------------------
// Cross-spectrum of partition p per channel, one-sided bins: G_c[k] = sum_{b >= p} Y0_c[b][k]
// conj(X_c[b - p][k]), scaled by 1 / 4096. A thread owns one bin of one slot and kCrossTile
// partitions: the input spectra enter a register ring one block per step (as in the product),
// the block's Y0 is read once for the whole tile. Each group of kCrossTile consecutive blocks is
// summed in float (at most kCrossTile terms), the groups in double, in block order.
constexpr int kCrossTile = 11;

__global__ __launch_bounds__(kBinWave) void rv_cross_kernel(int nb, int parts, const float4* Y0,
                                                            const float4* X, float4* Gs) {
  const int k = blockIdx.x * kBinWave + threadIdx.x;
  const int p0 = blockIdx.y * kCrossTile, slot = blockIdx.z;
  if (k > kN / 2) return;
  const float4* ys = Y0 + (int64_t)slot * nb * kRvStride + k;
  const float4* xs = X + (int64_t)slot * nb * kRvStride + k;
  const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 ring[kCrossTile];
  double acc[kCrossTile][4];
#pragma unroll
  for (int i = 0; i < kCrossTile; ++i) {
    ring[i] = zero;
    acc[i][0] = acc[i][1] = acc[i][2] = acc[i][3] = 0.0;
  }
  for (int b0 = 0; b0 < nb; b0 += kCrossTile) {
    float4 part[kCrossTile];
#pragma unroll
    for (int i = 0; i < kCrossTile; ++i) part[i] = zero;
#pragma unroll
    for (int j = 0; j < kCrossTile; ++j) {
      const int b = b0 + j;
      if (b < nb) {  // uniform
      const float4 xv = xs[(int64_t)max(b - p0, 0) * kRvStride];
      ring[j] = b - p0 >= 0 ? xv : zero;  // X[b - p0]
      const float4 y = ys[(int64_t)b * kRvStride];
#pragma unroll
      for (int i = 0; i < kCrossTile; ++i) {  // partition p0 + i: X[b - p0 - i]
        const float4 x = ring[(j - i + kCrossTile) % kCrossTile];
        part[i].x = fma(y.x, x.x, fma(y.y, x.y, part[i].x));
        part[i].y = fma(y.y, x.x, fma(-y.x, x.y, part[i].y));
        part[i].z = fma(y.z, x.z, fma(y.w, x.w, part[i].z));
        part[i].w = fma(y.w, x.z, fma(-y.z, x.w, part[i].w));
      }
      }
    }
#pragma unroll
    for (int i = 0; i < kCrossTile; ++i) {
      acc[i][0] += part[i].x;
      acc[i][1] += part[i].y;
      acc[i][2] += part[i].z;
      acc[i][3] += part[i].w;
    }
  }
  constexpr double s = 1.0 / kN;
#pragma unroll
  for (int i = 0; i < kCrossTile; ++i)
    if (p0 + i < parts)
      Gs[((int64_t)slot * parts + p0 + i) * kRvStride + k] =
          make_float4((float)(s * acc[i][0]), (float)(s * acc[i][1]), (float)(s * acc[i][2]),
                      (float)(s * acc[i][3]));
}

// hbar_c[2048 p + i] = first half of the inverse transform of G (left: real part, right:
// imaginary part of the packed transform G_l + i G_r). Lags from valid_len[slot] + valid_shift on
// have no term (the shifted signals no longer overlap) and are written as exact zeros, not as
// rounding residue; valid_len is the node's own length, so a node of a merged batch gets the
// bits it gets alone.
__global__ __launch_bounds__(kBlock) void rv_hbar_kernel(const float4* Gs, int parts, int64_t L,
                                                         const int32_t* valid_len, int valid_shift,
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
  const int64_t valid = (int64_t)valid_len[slot] + valid_shift;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int64_t n = (int64_t)kB * p + j + 256 * r;
    if (n < L) {
      hb[n] = n < valid ? v[r].x : 0.f;
      hb[L + n] = n < valid ? v[r].y : 0.f;
    }
  }
}

// Mask gradient. Frame m of channel x (mid, side) reads fbar[q] = hbar_x[192 m - 192 + q]
// (hbar_m = (hbar_l + hbar_r) / 2, hbar_s = (hbar_l - hbar_r) / 2), and the gradient with respect
// to the log-mask entry (k, m) is (c_k / 384) Re(Un[k] V_m[k]) mu[k] with
// V_m[k] = sum_q fbar[q] e^(2 pi i k q / 384) = D_{m-1}[k] + (-1)^k D_m[k], where
// D_s[k] = sum_{t<192} hbar_x[192 s + t] e^(2 pi i k t / 384) is the DFT of one hop segment. A
// block takes kGradFrames frames of one reverb slot: the kGradFrames + 1 segments it needs (both
// channels) in LDS, thread k - 1 forms D_s[k] of all of them for one bin k = 1..192 (the twiddle
// stepped by multiplication, restarted exactly every 64 samples; the DC bin is a plain sum), then
// the frames' gradients, summed into (sum_m G, sum_m m G) per bin in frame order. Per-block
// partials: part[slot][block][x][k] = (a, d).
constexpr int kGradFrames = 8;
constexpr int kGradSegs = kGradFrames + 1;

__global__ __launch_bounds__(kHop) void rv_mask_grad_kernel(const float* P, const double2* Un,
                                                            const float* hbar, int64_t L, int M,
                                                            double2* part) {
  __shared__ double2 seg[kGradSegs][kHop];  // (mid, side) per sample
  __shared__ double dc[kGradSegs][2];
  const int blk = blockIdx.x, slot = blockIdx.y, nblk = gridDim.x;
  const int m0 = blk * kGradFrames;
  const float* hb = hbar + (int64_t)slot * 2 * L;
  for (int i = threadIdx.x; i < kGradSegs * kHop; i += kHop) {
    const int j = i / kHop, t = i % kHop;
    const int64_t n = (int64_t)kHop * (m0 - 1 + j) + t;  // segment s = m0 - 1 + j
    double2 v = make_double2(0.0, 0.0);
    if (n >= 0 && n < L) {
      const double l = hb[n], r = hb[L + n];
      v = make_double2(0.5 * (l + r), 0.5 * (l - r));
    }
    seg[j][t] = v;
  }
  __syncthreads();
  if (threadIdx.x < 2 * kGradSegs) {  // the DC bin: plain sums
    const int j = threadIdx.x >> 1, x = threadIdx.x & 1;
    double a = 0.0;
    for (int t = 0; t < kHop; ++t) a += x ? seg[j][t].y : seg[j][t].x;
    dc[j][x] = a;
  }
  const int k = threadIdx.x + 1;  // 1..192
  double dr[kGradSegs][2], di[kGradSegs][2];
#pragma unroll
  for (int j = 0; j < kGradSegs; ++j) dr[j][0] = dr[j][1] = di[j][0] = di[j][1] = 0.0;
  double sr, si;
  sincospi(2.0 * k / kF, &si, &sr);
  for (int t0 = 0; t0 < kHop; t0 += 64) {
    double wr, wi;
    sincospi(2.0 * (double)((k * t0) % kF) / kF, &wi, &wr);
    for (int t = t0; t < t0 + 64; ++t) {
#pragma unroll
      for (int j = 0; j < kGradSegs; ++j) {
        const double2 v = seg[j][t];
        dr[j][0] = fma(v.x, wr, dr[j][0]);
        di[j][0] = fma(v.x, wi, di[j][0]);
        dr[j][1] = fma(v.y, wr, dr[j][1]);
        di[j][1] = fma(v.y, wi, di[j][1]);
      }
      const double tt = wr * sr - wi * si;
      wi = fma(wr, si, wi * sr);
      wr = tt;
    }
  }
  __syncthreads();  // dc ready
  const float* p = P + (int64_t)slot * kRvParams;
  double2* out = part + ((int64_t)slot * nblk + blk) * 2 * kK;
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    double a = 0.0, d = 0.0, a0 = 0.0, d0 = 0.0;
    const double sg = (k & 1) ? -1.0 : 1.0;
    const double ck = (k == kK - 1) ? 1.0 / kF : 2.0 / kF;
#pragma unroll
    for (int f = 0; f < kGradFrames; ++f) {
      const int m = m0 + f;
      if (m >= M) break;
      const double vr = dr[f][x] + sg * dr[f + 1][x], vi = di[f][x] + sg * di[f + 1][x];
      const double2 u = Un[((int64_t)x * M + m) * kK + k];
      const double g = ck * (u.x * vr - u.y * vi) * mask_at(p, x, k, m);
      a += g;
      d = fma((double)m, g, d);
      if (threadIdx.x == 0) {  // the DC bin
        const double2 u0 = Un[((int64_t)x * M + m) * kK];
        const double g0 = (1.0 / kF) * (u0.x * (dc[f][x] + dc[f + 1][x])) * mask_at(p, x, 0, m);
        a0 += g0;
        d0 = fma((double)m, g0, d0);
      }
    }
    out[x * kK + k] = make_double2(a, d);
    if (threadIdx.x == 0) out[x * kK] = make_double2(a0, d0);
  }
}

// dH0[k] = sum_m G[m][k], dHD[k] = sum_m m G[m][k]: the blocks' partials in block order (bin 191
// adds the Nyquist bin, which shares its mask).
__global__ __launch_bounds__(kBlock) void rv_param_grad_kernel(const double2* part, int nblk,
                                                               float* dP) {
  const int slot = blockIdx.x, x = blockIdx.y, k = threadIdx.x;
  if (k >= kRvBins) return;
  double a = 0.0, d = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double2* pb = part + (((int64_t)slot * nblk + b) * 2 + x) * kK;
    double2 v = pb[k];
    if (k == kRvBins - 1) {
      const double2 w = pb[kK - 1];
      v.x += w.x;
      v.y += w.y;
    }
    a += v.x;
    d += v.y;
  }
  float* out = dP + (int64_t)slot * kRvParams + x * 2 * kRvBins;
  out[k] = (float)a;
  out[kRvBins + k] = (float)d;
}

}  // namespace

int rv_frames(int64_t L) { return (int)((L + kHop - 1) / kHop) + 1; }
int rv_parts(int64_t L) { return (int)((L + kB - 1) / kB); }
int rv_blocks(int64_t T) { return (int)((T + kB - 1) / kB); }
int rv_grad_blocks(int64_t L) { return (rv_frames(L) + kGradFrames - 1) / kGradFrames; }

hipError_t launch_rv_design(const float* P, int n, const float* noise, int64_t L, double2* Un,
                            float* h, float4* Hs, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int M = rv_frames(L), parts = rv_parts(L);
  rv_noise_stft_kernel<<<dim3(M, 2), kBlock, 0, s>>>(noise, L, M, Un);
  rv_ir_kernel<<<dim3((M - 1 + kIrHops - 1) / kIrHops, n), kIrThreads, 0, s>>>(P, Un, L, M, h);
  rv_partition_kernel<<<dim3(parts, n), kBlock, 0, s>>>(h, L, parts, Hs);
  return hipGetLastError();
}

hipError_t launch_xcorr_spectra(const GraphView& g, int node_begin, int n_nodes, bool adj,
                                int shift, int nb, float4* out, int32_t* slot_len, hipStream_t s) {
  if (adj)
    rv_spectra_kernel<true><<<dim3(nb, n_nodes), kBlock, 0, s>>>(g, node_begin, nb, shift, out,
                                                                 slot_len);
  else
    rv_spectra_kernel<false><<<dim3(nb, n_nodes), kBlock, 0, s>>>(g, node_begin, nb, shift, out,
                                                                  slot_len);
  return hipGetLastError();
}

hipError_t launch_xcorr(int n, int nb, int parts, int64_t len, const int32_t* valid_len,
                        int valid_shift, const float4* Y0, const float4* X, float4* Gs, float* R,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  rv_cross_kernel<<<dim3(kBinWaves, (parts + kCrossTile - 1) / kCrossTile, n), kBinWave, 0, s>>>(
      nb, parts, Y0, X, Gs);
  rv_hbar_kernel<<<dim3(parts, n), kBlock, 0, s>>>(Gs, parts, len, valid_len, valid_shift, R);
  return hipGetLastError();
}

int rv_conv_tiles(int64_t L) { return (rv_parts(L) + kConvTile - 1) / kConvTile; }

hipError_t launch_rv_fwd(const GraphView& g, float* U, int node_begin, int n_nodes, int64_t L,
                         const float4* Hs, float4* Z, float4* C, hipStream_t s) {
  const int nb = rv_blocks(g.T), parts = rv_parts(L), tiles = rv_conv_tiles(L);
  rv_spectra_kernel<false><<<dim3(nb, n_nodes), kBlock, 0, s>>>(g, node_begin, nb, 0, Z, nullptr);
  const int nseg = (nb + kConvSeg - 1) / kConvSeg;
  rv_conv_bins_kernel<false><<<dim3(kBinWaves, tiles * nseg, n_nodes), kBinWave, 0, s>>>(
      g, node_begin, nb, parts, tiles, nseg, Z, Hs, C);
  rv_inverse_kernel<false><<<dim3(nb, n_nodes), kBlock, 0, s>>>(g, U, node_begin, nb, tiles, C);
  return hipGetLastError();
}

hipError_t launch_rv_bwd(const GraphView& g, float* dU, int node_begin, int n_nodes, int64_t L,
                         const float4* Hs, float4* Y0, float4* C, int32_t* slot_len,
                         hipStream_t s) {
  const int nb = rv_blocks(g.T), parts = rv_parts(L), tiles = rv_conv_tiles(L);
  rv_spectra_kernel<true><<<dim3(nb, n_nodes), kBlock, 0, s>>>(g, node_begin, nb, 0, Y0, slot_len);
  const int nseg = (nb + kConvSeg - 1) / kConvSeg;
  rv_conv_bins_kernel<true><<<dim3(kBinWaves, tiles * nseg, n_nodes), kBinWave, 0, s>>>(
      g, node_begin, nb, parts, tiles, nseg, Y0, Hs, C);
  rv_inverse_kernel<true><<<dim3(nb, n_nodes), kBlock, 0, s>>>(g, dU, node_begin, nb, tiles, C);
  return hipGetLastError();
}

hipError_t launch_rv_grad(int n, int64_t T, int64_t L, const float* P, const double2* Un,
                          const float4* Z, const float4* Y0, const int32_t* slot_len, float4* Gs,
                          float* hbar, double* part, float* dP, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nb = rv_blocks(T), parts = rv_parts(L), M = rv_frames(L);
  // hbar[n] = sum_t ybar[t] u[t - n] has no term for n >= the node's length
  const hipError_t e = launch_xcorr(n, nb, parts, L, slot_len, 0, Y0, Z, Gs, hbar, s);
  if (e != hipSuccess) return e;
  const int nblk = rv_grad_blocks(L);
  rv_mask_grad_kernel<<<dim3(nblk, n), kHop, 0, s>>>(P, Un, hbar, L, M,
                                                     reinterpret_cast<double2*>(part));
  rv_param_grad_kernel<<<dim3(n, 2), kBlock, 0, s>>>(reinterpret_cast<const double2*>(part),
                                                     nblk, dP);
  return hipGetLastError();
}

}  // namespace grafx
