// Multi-resolution STFT loss and its adjoint (the loss of the gradient-descent mixing
// application, paper Sec. 4): resolutions 512, 1024, 2048, hop r/4, periodic Hann window,
// frames inside [0, T), S = sqrt(|X|^2 + 1e-8),
// L = (1/3) sum_r ( ||S_y - S_t||_F / ||S_t||_F + mean |ln S_y - ln S_t| ).
//
// A group of G threads per frame (one wave for N = 512 and 1024, two waves for N = 2048), several
// frames per block. Both channels of a frame ride in one complex FFT (left + i right) held in
// registers, N/G points per thread: one radix-N/G pass in registers, then two passes whose
// radices multiply to G, exchanging through the group's own LDS slice; a one-wave group needs no
// block-wide barrier. The two spectra of a frame (output and target) are kept in LDS, where the
// channel spectra are separated through conjugate symmetry (bins k and N - k).
// Per-block partial sums (double) are reduced in a fixed order by a single block. The adjoint
// rebuilds each frame's spectra, forms dL/dX per bin, assembles the Hermitian spectrum whose
// inverse transform is the windowed frame gradient (again both channels in one complex
// transform), and an overlap-add pass sums, for every sample, the frames that cover it in a
// fixed order.
#include "device_common.h"
#include "grafx_internal.h"
#include "kernels.h"
#include "tables.inc"

namespace grafx {
namespace {

constexpr float kMagEps = 1e-8f;
constexpr int kRes[3] = {512, 1024, 2048};
constexpr int kWaves = kBlock / 64;

int frames_of(int64_t T, int r) { return T >= r ? (int)((T - r) / (r / 4) + 1) : 0; }
int frames_per_block(int r) { return r == 2048 ? kBlock / 128 : kBlock / 64; }
int blocks_of(int64_t T, int r) {
  return (frames_of(T, r) + frames_per_block(r) - 1) / frames_per_block(r);
}

struct Layout {
  size_t consts;     // double [3][2]: (c_sc, c_lm) per resolution
  size_t part[3];    // double [blocks_r * rows][3]
  size_t fb[3];      // float [rows][F_r][2][r] frame gradients
  size_t total;
};

Layout layout(int rows, int64_t T) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  L.consts = take(8 * sizeof(double));
  for (int i = 0; i < 3; ++i)
    L.part[i] = take((size_t)blocks_of(T, kRes[i]) * rows * 3 * sizeof(double));
  for (int i = 0; i < 3; ++i)
    L.fb[i] = take((size_t)rows * frames_of(T, kRes[i]) * 2 * kRes[i] * sizeof(float));
  L.total = off;
  return L;
}

// exp(-+2 pi i q / N), q in [0, N)
template <int N, bool INV>
__device__ __forceinline__ float2 twid(int q) {
  const float2 w = kTw4096[q * (4096 / N)];
  return INV ? make_float2(w.x, -w.y) : w;
}

__device__ __forceinline__ constexpr int lpad(int i) { return i + (i >> 4); }

// LDS accesses of one wave are executed in order; this keeps the compiler from moving them across
// a phase boundary of the wave's exchange and waits for the wave's outstanding LDS operations.
__device__ __forceinline__ void wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <bool INV>
__device__ __forceinline__ void dft32(float2* v) {
  // 32 = 2 x 16: n = 2 n1 + n2, k = k1 + 16 k2
  float2 e[16], o[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    e[i] = v[2 * i];
    o[i] = v[2 * i + 1];
  }
  dft16<INV>(e);
  dft16<INV>(o);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float2 t = k == 0 ? o[0] : cmul(o[k], twid<32, INV>(k));
    v[k] = cadd(e[k], t);
    v[k + 16] = csub(e[k], t);
  }
}

template <int P, bool INV>
__device__ __forceinline__ void dft_p(float2* v) {
  if constexpr (P == 32) dft32<INV>(v);
  else dft_r<P, INV>(v);
}

// Threads per frame and the first cross-thread radix for each resolution.
template <int N> struct Grp { static constexpr int G = 64, R1 = 8; };
template <> struct Grp<2048> { static constexpr int G = 128, R1 = 16; };

// Exchange boundary of a group: a one-wave group only orders its own LDS accesses; larger groups
// synchronise the block (all groups of a block run the same code path).
template <int G>
__device__ __forceinline__ void group_sync() {
  if constexpr (G == 64) wave_sync();
  else __syncthreads();
}

// In-place N-point DFT over a group of G threads (forward exp(-2 pi i nk/N), inverse exp(+...),
// unnormalised). On entry v[m] holds x[j + G m] for thread j of the group; on exit X[j + G m].
// s: the group's LDS slice of lpad(N - 1) + 1 entries. Stockham passes: radix P = N/G
// (sub-transform size 1), radix R1 (size P), radix R2 = G/R1 (size P R1).
template <int N, bool INV>
__device__ __forceinline__ void group_fft(float2 (&v)[N / Grp<N>::G], float2* s, int j) {
  constexpr int G = Grp<N>::G, P = N / G, R1 = Grp<N>::R1, R2 = G / R1;
  static_assert(P % R1 == 0 && P % R2 == 0, "radices must divide the points per thread");
  dft_p<P, INV>(v);
#pragma unroll
  for (int r = 0; r < P; ++r) s[lpad(P * j + r)] = v[r];
  group_sync<G>();
  {  // butterflies b = j + G h, inputs b + (N/R1) r, twiddles exp(-+2 pi i r (b mod P) / (R1 P))
#pragma unroll
    for (int h = 0; h < P / R1; ++h)
#pragma unroll
      for (int r = 0; r < R1; ++r) v[R1 * h + r] = s[lpad(j + G * h + (N / R1) * r)];
    group_sync<G>();
    const int k = j % P;
    float2 w[R1];
#pragma unroll
    for (int r = 1; r < R1; ++r) w[r] = twid<N, INV>(r * k * (N / (R1 * P)));
#pragma unroll
    for (int h = 0; h < P / R1; ++h) {
      float2* u = v + R1 * h;
#pragma unroll
      for (int r = 1; r < R1; ++r) u[r] = cmul(u[r], w[r]);
      dft_r<R1, INV>(u);
      const int b = j + G * h;
      const int base = (b / P) * P * R1 + k;
#pragma unroll
      for (int r = 0; r < R1; ++r) s[lpad(base + P * r)] = u[r];
    }
    group_sync<G>();
  }
  {  // butterflies b = j + G h, inputs b + (N/R2) r, twiddles exp(-+2 pi i r b / N)
#pragma unroll
    for (int h = 0; h < P / R2; ++h)
#pragma unroll
      for (int r = 0; r < R2; ++r) v[R2 * h + r] = s[lpad(j + G * h + (N / R2) * r)];
    group_sync<G>();
    float2 o[P];
#pragma unroll
    for (int h = 0; h < P / R2; ++h) {
      float2* u = v + R2 * h;
      const int b = j + G * h;
#pragma unroll
      for (int r = 1; r < R2; ++r) u[r] = cmul(u[r], twid<N, INV>(r * b));
      dft_r<R2, INV>(u);
#pragma unroll
      for (int r = 0; r < R2; ++r) o[h + (P / R2) * r] = u[r];  // X[j + G (h + (P/R2) r)]
    }
#pragma unroll
    for (int m = 0; m < P; ++m) v[m] = o[m];
  }
}

template <int N>
__device__ __forceinline__ float hann(int n) {
  return 0.5f - 0.5f * kTw4096[n * (4096 / N)].x;
}

// Forward transform of one windowed stereo frame (left + i right) by thread j of its group; the
// spectrum is left in s at lpad(k).
template <int N>
__device__ __forceinline__ void frame_spectrum(const float* row, int64_t T, int64_t s0, float2* s,
                                               int j) {
  constexpr int G = Grp<N>::G, P = N / G;
  float2 v[P];
#pragma unroll
  for (int m = 0; m < P; ++m) {
    const int n = j + G * m;
    const float w = hann<N>(n);
    v[m] = make_float2(w * row[s0 + n], w * row[T + s0 + n]);
  }
  group_fft<N, false>(v, s, j);
  group_sync<G>();
#pragma unroll
  for (int m = 0; m < P; ++m) s[lpad(j + G * m)] = v[m];
}

// Separate the spectra of the two real channels from Z = FFT(l + i r).
__device__ __forceinline__ void split(float2 zk, float2 znk, float2& xl, float2& xr) {
  xl = make_float2(0.5f * (zk.x + znk.x), 0.5f * (zk.y - znk.y));
  xr = make_float2(0.5f * (zk.y + znk.y), -0.5f * (zk.x - znk.x));
}

// Per-bin arithmetic is in float (the spectra themselves are float); sums are kept in double.
__device__ __forceinline__ float mag(float2 x) {
  return sqrtf(fmaf(x.x, x.x, fmaf(x.y, x.y, kMagEps)));
}

// Bins k = j + G i of thread j (i < N/(2G)), and bin N/2 on thread 0: every bin of [0, N/2] once.
template <int N, typename F>
__device__ __forceinline__ void for_half_bins(int j, F&& fn) {
  constexpr int G = Grp<N>::G;
#pragma unroll 2
  for (int i = 0; i < N / (2 * G); ++i) fn(j + G * i);
  if (j == 0) fn(N / 2);
}

// LDS of one block of the statistics and gradient passes: FPB frames x (output, target) spectra
template <int N>
constexpr int lds_entries() {
  return (kBlock / Grp<N>::G) * 2 * (lpad(N - 1) + 1);
}
constexpr int kLdsMax = lds_entries<2048>() > lds_entries<1024>()
                            ? (lds_entries<2048>() > lds_entries<512>() ? lds_entries<2048>()
                                                                        : lds_entries<512>())
                            : (lds_entries<1024>() > lds_entries<512>() ? lds_entries<1024>()
                                                                        : lds_entries<512>());

// Statistics of the frames of block bx of resolution N (one of the fused launch's ranges).
template <int N>
__device__ __forceinline__ void stats_body(int bx, int rows, int64_t T, int frames, const float* Y,
                                           const float* tgt, double* part, float2* lds,
                                           double (*red)[3]) {
  constexpr int G = Grp<N>::G, FPB = kBlock / G, S = lpad(N - 1) + 1;
  const int grp = (int)threadIdx.x / G, j = (int)threadIdx.x % G;
  const int f = bx * FPB + grp, row = blockIdx.y;
  const bool live = f < frames;  // uniform over the group
  double acc[3] = {0.0, 0.0, 0.0};  // sum (S_y - S_t)^2, sum S_t^2, sum |ln S_y - ln S_t|
  if (G == 64 ? live : true) {  // multi-wave groups keep every barrier convergent
    float2* sy = lds + grp * 2 * S;
    float2* st = sy + S;
    const int64_t s0 = (int64_t)(live ? f : frames - 1) * (N / 4);
    frame_spectrum<N>(Y + (int64_t)row * 2 * T, T, s0, sy, j);
    frame_spectrum<N>(tgt + (int64_t)row * 2 * T, T, s0, st, j);
    group_sync<G>();
    if (live)
      for_half_bins<N>(j, [&](int k) {
        const int nk = (N - k) & (N - 1);
        float2 yl, yr, tl, tr;
        split(sy[lpad(k)], sy[lpad(nk)], yl, yr);
        split(st[lpad(k)], st[lpad(nk)], tl, tr);
        const float my[2] = {mag(yl), mag(yr)}, mt[2] = {mag(tl), mag(tr)};
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int ch = 0; ch < 2; ++ch) {
          const float d = my[ch] - mt[ch];
          a0 = fmaf(d, d, a0);
          a1 = fmaf(mt[ch], mt[ch], a1);
          a2 += fabsf(logf(my[ch]) - logf(mt[ch]));
        }
        acc[0] += (double)a0;
        acc[1] += (double)a1;
        acc[2] += (double)a2;
      });
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < 3; ++q) acc[q] = wave_sum<double>(acc[q]);
  if (l == 0)
#pragma unroll
    for (int q = 0; q < 3; ++q) red[w][q] = acc[q];
  __syncthreads();
  if (threadIdx.x < 3) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) v += red[q][threadIdx.x];
    part[((int64_t)bx * rows + row) * 3 + threadIdx.x] = v;
  }
}

struct Frames {
  int F[3], B[3];
  double* part[3];
};

// Fixed-order reduction of the per-block partial sums of all three resolutions.
__global__ __launch_bounds__(kBlock) void reduce_kernel(int rows, Frames fr, double* consts,
                                                        float* loss) {
  __shared__ double red[kWaves][9];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  double s[9];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const int n = fr.B[i] * rows;
    for (int q = threadIdx.x; q < n; q += kBlock) {
      a0 += fr.part[i][(int64_t)q * 3];
      a1 += fr.part[i][(int64_t)q * 3 + 1];
      a2 += fr.part[i][(int64_t)q * 3 + 2];
    }
    s[3 * i] = wave_sum<double>(a0);
    s[3 * i + 1] = wave_sum<double>(a1);
    s[3 * i + 2] = wave_sum<double>(a2);
  }
  if (l == 0)
#pragma unroll
    for (int j = 0; j < 9; ++j) red[w][j] = s[j];
  __syncthreads();
  if (threadIdx.x != 0) return;
  double L = 0.0;
  for (int i = 0; i < 3; ++i) {
    double t[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < kWaves; ++q)
      for (int j = 0; j < 3; ++j) t[j] += red[q][3 * i + j];
    const int n = fr.F[i] * rows;
    if (n > 0) {
      const double nd = sqrt(t[0]), nt = sqrt(t[1]);
      const double M = (double)n * 2.0 * (kRes[i] / 2 + 1);
      L += nd / nt + t[2] / M;
      consts[2 * i] = nd > 0.0 ? 1.0 / (3.0 * nd * nt) : 0.0;
      consts[2 * i + 1] = 1.0 / (3.0 * M);
    } else {
      consts[2 * i] = consts[2 * i + 1] = 0.0;
    }
  }
  *loss = (float)(L / 3.0);
}

// Frame gradients of block bx of resolution N (one of the fused launch's ranges).
template <int N>
__device__ __forceinline__ void grad_body(int bx, int rows, int64_t T, int frames, const float* Y,
                                          const float* tgt, const double* consts, int res,
                                          const float* dloss, float* fb, float2* lds) {
  constexpr int G = Grp<N>::G, FPB = kBlock / G, P = N / G, S = lpad(N - 1) + 1;
  const int grp = (int)threadIdx.x / G, j = (int)threadIdx.x % G;
  const int f = bx * FPB + grp, row = blockIdx.y;
  const bool live = f < frames;  // uniform over the group
  if (G == 64 && !live) return;  // one-wave groups need no block-wide barrier
  float2* sy = lds + grp * 2 * S;
  float2* st = sy + S;
  const int64_t s0 = (int64_t)(live ? f : frames - 1) * (N / 4);
  frame_spectrum<N>(Y + (int64_t)row * 2 * T, T, s0, sy, j);
  frame_spectrum<N>(tgt + (int64_t)row * 2 * T, T, s0, st, j);
  group_sync<G>();
  const double up = (double)*dloss;
  const float c_sc = (float)(consts[2 * res] * up), c_lm = (float)(consts[2 * res + 1] * up);
  // Hermitian spectrum of the frame gradient, both channels packed (F = F_l + i F_r), written
  // over sy: the pair {k, N - k} is read and written by one thread only.
  for_half_bins<N>(j, [&](int k) {
    const int nk = (N - k) & (N - 1);
    float2 x[2], tt[2];
    split(sy[lpad(k)], sy[lpad(nk)], x[0], x[1]);
    split(st[lpad(k)], st[lpad(nk)], tt[0], tt[1]);
    float2 Gc[2];
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      const float my = mag(x[ch]), mt = mag(tt[ch]);
      const float dl = logf(my) - logf(mt);
      const float sgn = dl > 0.f ? 1.f : (dl < 0.f ? -1.f : 0.f);
      const float inv = 1.f / my;
      const float gS = fmaf(c_sc, my - mt, c_lm * sgn * inv) * inv;
      Gc[ch] = make_float2(gS * x[ch].x, gS * x[ch].y);
    }
    if (k == 0 || k == N / 2) {
      sy[lpad(k)] = make_float2(Gc[0].x, Gc[1].x);
    } else {
      const float2 gl = make_float2(0.5f * Gc[0].x, 0.5f * Gc[0].y);
      const float2 gr = make_float2(0.5f * Gc[1].x, 0.5f * Gc[1].y);
      sy[lpad(k)] = make_float2(gl.x - gr.y, gl.y + gr.x);
      sy[lpad(nk)] = make_float2(gl.x + gr.y, -gl.y + gr.x);  // conj(gl) + i conj(gr)
    }
  });
  group_sync<G>();
  float2 v[P];
#pragma unroll
  for (int m = 0; m < P; ++m) v[m] = sy[lpad(j + G * m)];
  group_sync<G>();
  group_fft<N, true>(v, st, j);
  if (!live) return;
  float* out = fb + ((int64_t)row * frames + f) * 2 * N;
#pragma unroll
  for (int m = 0; m < P; ++m) {
    const int n = j + G * m;
    const float wn = hann<N>(n);
    out[n] = wn * v[m].x;
    out[N + n] = wn * v[m].y;
  }
}

struct FrameBufs {
  int F[3];
  const float* fb[3];
};

// One launch for the three resolutions: block ranges [2048 | 1024 | 512] (the heaviest first),
// each block running the code of its range with the largest range's LDS.
__global__ __launch_bounds__(kBlock) void stats_all_kernel(int rows, int64_t T, Frames fr,
                                                           const float* Y, const float* tgt) {
  __shared__ float2 lds[kLdsMax];
  __shared__ double red[kWaves][3];
  int bx = blockIdx.x;
  if (bx < fr.B[2]) {
    stats_body<2048>(bx, rows, T, fr.F[2], Y, tgt, fr.part[2], lds, red);
    return;
  }
  bx -= fr.B[2];
  if (bx < fr.B[1]) {
    stats_body<1024>(bx, rows, T, fr.F[1], Y, tgt, fr.part[1], lds, red);
    return;
  }
  stats_body<512>(bx - fr.B[1], rows, T, fr.F[0], Y, tgt, fr.part[0], lds, red);
}

struct GradArgs {
  int F[3], B[3];
  float* fb[3];
};

__global__ __launch_bounds__(kBlock) void grad_all_kernel(int rows, int64_t T, GradArgs ga,
                                                          const float* Y, const float* tgt,
                                                          const double* consts,
                                                          const float* dloss) {
  __shared__ float2 lds[kLdsMax];
  int bx = blockIdx.x;
  if (bx < ga.B[2]) {
    grad_body<2048>(bx, rows, T, ga.F[2], Y, tgt, consts, 2, dloss, ga.fb[2], lds);
    return;
  }
  bx -= ga.B[2];
  if (bx < ga.B[1]) {
    grad_body<1024>(bx, rows, T, ga.F[1], Y, tgt, consts, 1, dloss, ga.fb[1], lds);
    return;
  }
  grad_body<512>(bx - ga.B[1], rows, T, ga.F[0], Y, tgt, consts, 0, dloss, ga.fb[0], lds);
}

__global__ __launch_bounds__(kBlock) void ola_kernel(int rows, int64_t T, FrameBufs fbs,
                                                     float* dY) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= (int64_t)rows * 2 * T) return;
  const int64_t t = idx % T;
  const int64_t rc = idx / T;  // row * 2 + channel
  const int row = (int)(rc >> 1), ch = (int)(rc & 1);
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int r = kRes[i], h = r / 4, F = fbs.F[i];
    if (F == 0) continue;
    const int64_t fmin = t < r ? 0 : (t - r) / h + 1;
    const int64_t fmax = min((int64_t)F - 1, t / h);
    for (int64_t f = fmin; f <= fmax; ++f)
      acc += fbs.fb[i][(((int64_t)row * F + f) * 2 + ch) * r + (t - f * h)];
  }
  dY[idx] = acc;
}


// ---- log-mel features of the learned initialiser -----------------------------------------------
// Frames of 1024 samples at hop 256 inside [0, T), periodic Hann window; one group of 64 threads
// per frame transforms left + i right, separates the channel spectra and forms the power of their
// mean (the mono signal); 128 triangular filters on the HTK mel scale (130 edges evenly spaced in
// mel over [0, fs/2], filter b rising from edge b to b + 1 and falling to b + 2, peak 1) sum the
// power, and the feature is (ln(E + 1e-6) + 5) / 5.
constexpr int kMels = 128;
constexpr float kFs = 44100.f;

__device__ __forceinline__ float mel_edge_hz(int e) {
  const float top = 2595.f * log10f(1.f + 0.5f * kFs / 700.f);
  return 700.f * (exp10f(top * (float)e / (float)(kMels + 1) / 2595.f) - 1.f);
}

__global__ __launch_bounds__(kBlock) void logmel_kernel(int64_t T, int frames, const float* sig,
                                                        float* feats) {
  constexpr int N = 1024, G = Grp<N>::G, FPB = kBlock / G, S = lpad(N - 1) + 1;
  __shared__ float2 lds[FPB * S];
  const int grp = (int)threadIdx.x / G, j = (int)threadIdx.x % G;
  const int f = blockIdx.x * FPB + grp, row = blockIdx.y;
  if (f >= frames) return;  // whole one-wave group: no block barrier below
  float2* s = lds + grp * S;
  frame_spectrum<N>(sig + (int64_t)row * 2 * T, T, (int64_t)f * (N / 4), s, j);
  group_sync<G>();
  constexpr int NB = N / (2 * G);  // bins j + G i, i < NB, per thread; bin N/2 on thread 0
  float pw[NB + 1];
#pragma unroll
  for (int i = 0; i <= NB; ++i) {
    const int k = i < NB ? j + G * i : N / 2;
    float2 xl, xr;
    split(s[lpad(k)], s[lpad((N - k) & (N - 1))], xl, xr);
    const float re = 0.5f * (xl.x + xr.x), im = 0.5f * (xl.y + xr.y);
    pw[i] = fmaf(re, re, im * im);
  }
  group_sync<G>();
  float* P = reinterpret_cast<float*>(s);
#pragma unroll
  for (int i = 0; i < NB; ++i) P[j + G * i] = pw[i];
  if (j == 0) P[N / 2] = pw[NB];
  group_sync<G>();
  constexpr float kBinHz = kFs / N;
  for (int b = j; b < kMels; b += G) {
    const float lo = mel_edge_hz(b), mid = mel_edge_hz(b + 1), hi = mel_edge_hz(b + 2);
    const int k0 = max(0, (int)ceilf(lo / kBinHz)), k1 = min(N / 2, (int)floorf(hi / kBinHz));
    float e = 0.f;
    for (int k = k0; k <= k1; ++k) {
      const float fk = (float)k * kBinHz;
      const float wgt = fmaxf(0.f, fminf((fk - lo) / (mid - lo), (hi - fk) / (hi - mid)));
      e = fmaf(wgt, P[k], e);
    }
    feats[((int64_t)row * kMels + b) * frames + f] = (logf(e + 1e-6f) + 5.f) * 0.2f;
  }
}

}  // namespace

size_t mrstft_ws_bytes(int rows, int64_t T) { return layout(rows, T).total; }

hipError_t launch_mrstft_loss(int rows, int64_t T, const float* Y, const float* tgt, float* loss,
                              void* ws, hipStream_t s) {
  const Layout L = layout(rows, T);
  char* base = static_cast<char*>(ws);
  Frames fr;
  for (int i = 0; i < 3; ++i) {
    fr.F[i] = frames_of(T, kRes[i]);
    fr.B[i] = blocks_of(T, kRes[i]);
    fr.part[i] = reinterpret_cast<double*>(base + L.part[i]);
  }
  Frames run = fr;  // block ranges of the fused launch: none for a resolution without frames
  for (int i = 0; i < 3; ++i)
    if (run.F[i] <= 0) run.B[i] = 0;
  const int nb = run.B[0] + run.B[1] + run.B[2];
  if (nb > 0)
    stats_all_kernel<<<dim3(nb, rows), kBlock, 0, s>>>(rows, T, run, Y, tgt);
  reduce_kernel<<<1, kBlock, 0, s>>>(rows, fr, reinterpret_cast<double*>(base + L.consts), loss);
  return hipGetLastError();
}

hipError_t launch_mrstft_bwd(int rows, int64_t T, const float* Y, const float* tgt,
                             const float* dloss, float* dY, void* ws, hipStream_t s) {
  const Layout L = layout(rows, T);
  char* base = static_cast<char*>(ws);
  const double* consts = reinterpret_cast<const double*>(base + L.consts);
  FrameBufs fbs;
  for (int i = 0; i < 3; ++i) {
    fbs.F[i] = frames_of(T, kRes[i]);
    fbs.fb[i] = reinterpret_cast<const float*>(base + L.fb[i]);
  }
  float* fb0 = reinterpret_cast<float*>(base + L.fb[0]);
  float* fb1 = reinterpret_cast<float*>(base + L.fb[1]);
  float* fb2 = reinterpret_cast<float*>(base + L.fb[2]);
  GradArgs ga;
  float* fbw[3] = {fb0, fb1, fb2};
  for (int i = 0; i < 3; ++i) {
    ga.F[i] = fbs.F[i];
    ga.B[i] = fbs.F[i] > 0 ? blocks_of(T, kRes[i]) : 0;
    ga.fb[i] = fbw[i];
  }
  const int nb = ga.B[0] + ga.B[1] + ga.B[2];
  if (nb > 0)
    grad_all_kernel<<<dim3(nb, rows), kBlock, 0, s>>>(rows, T, ga, Y, tgt, consts, dloss);
  const int64_t n = (int64_t)rows * 2 * T;
  ola_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(rows, T, fbs, dY);
  return hipGetLastError();
}

hipError_t launch_logmel(int n_sig, int64_t T, const float* sig, float* feats, hipStream_t s) {
  const int frames = logmel_frames(T);
  if (n_sig <= 0 || frames <= 0) return hipSuccess;
  constexpr int FPB = kBlock / Grp<1024>::G;
  logmel_kernel<<<dim3((frames + FPB - 1) / FPB, n_sig), kBlock, 0, s>>>(T, frames, sig, feats);
  return hipGetLastError();
}

int logmel_frames(int64_t T) { return T >= 1024 ? (int)((T - 1024) / 256 + 1) : 0; }

}  // namespace grafx
