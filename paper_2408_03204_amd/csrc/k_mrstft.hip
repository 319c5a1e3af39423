// Multi-resolution STFT loss and its adjoint (the loss of the gradient-descent mixing
// application, paper Sec. 4): resolutions 512, 1024, 2048, hop r/4, periodic Hann window,
// frames inside [0, T), S = sqrt(|X|^2 + 1e-8),
// L = (1/3) sum_r ( ||S_y - S_t||_F / ||S_t||_F + mean |ln S_y - ln S_t| ).
//
// One block per (frame, row, resolution): both channels of a frame ride in one complex FFT
// (left + i right) and are separated through conjugate symmetry; per-block partial sums (double)
// are reduced in a fixed order by a single block. The adjoint rebuilds each frame's spectra,
// forms dL/dX per bin, assembles the Hermitian spectrum whose inverse transform is the windowed
// frame gradient (again both channels in one complex transform), and an overlap-add pass sums,
// for every sample, the frames that cover it in a fixed order.
#include "device_common.h"
#include "grafx_internal.h"
#include "kernels.h"
#include "tables.inc"

namespace grafx {
namespace {

constexpr double kMagEps = 1e-8;
constexpr int kRes[3] = {512, 1024, 2048};

int frames_of(int64_t T, int r) { return T >= r ? (int)((T - r) / (r / 4) + 1) : 0; }

struct Layout {
  size_t consts;     // double [3][2]: (c_sc, c_lm) per resolution; then loss parts
  size_t part[3];    // double [F_r * rows][3]
  size_t fb[3];      // float [rows][F_r][2][r] frame gradients
  size_t total;
};

Layout layout(int rows, int64_t T) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  L.consts = take(8 * sizeof(double));
  for (int i = 0; i < 3; ++i) L.part[i] = take((size_t)frames_of(T, kRes[i]) * rows * 3 * sizeof(double));
  for (int i = 0; i < 3; ++i)
    L.fb[i] = take((size_t)rows * frames_of(T, kRes[i]) * 2 * kRes[i] * sizeof(float));
  L.total = off;
  return L;
}

template <bool INV>
__device__ __forceinline__ float2 twid(int m) {
  const float2 w = kTw4096[m];
  return INV ? make_float2(w.x, -w.y) : w;
}

template <int N, int R, int NS, bool INV>
__device__ __forceinline__ void stockham_pass(const float2* in, float2* out) {
  constexpr int L = N / R;
  for (int j = threadIdx.x; j < L; j += kBlock) {
    const int k = j % NS;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[j + r * L];
    if (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twid<INV>(r * k * (4096 / (NS * R))));
    }
    dft_r<R, INV>(v);
    const int base = (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[base + r * NS] = v[r];
  }
  __syncthreads();
}

// Three-pass Stockham FFT in LDS: input in a, output in b (a is clobbered).
template <int N, bool INV>
__device__ __forceinline__ void lds_fft(float2* a, float2* b) {
  if constexpr (N == 512) {
    stockham_pass<N, 8, 1, INV>(a, b);
    stockham_pass<N, 8, 8, INV>(b, a);
    stockham_pass<N, 8, 64, INV>(a, b);
  } else if constexpr (N == 1024) {
    stockham_pass<N, 16, 1, INV>(a, b);
    stockham_pass<N, 16, 16, INV>(b, a);
    stockham_pass<N, 4, 256, INV>(a, b);
  } else {
    stockham_pass<N, 16, 1, INV>(a, b);
    stockham_pass<N, 16, 16, INV>(b, a);
    stockham_pass<N, 8, 256, INV>(a, b);
  }
}

template <int N>
__device__ __forceinline__ float hann(int n) {
  return 0.5f - 0.5f * kTw4096[n * (4096 / N)].x;
}

// Load one windowed stereo frame as left + i right.
template <int N>
__device__ __forceinline__ void load_frame(const float* row, int64_t T, int64_t s0, float2* a) {
  for (int n = threadIdx.x; n < N; n += kBlock) {
    const float w = hann<N>(n);
    a[n] = make_float2(w * row[s0 + n], w * row[T + s0 + n]);
  }
}

// Separate the spectra of the two real channels from Z = FFT(l + i r).
__device__ __forceinline__ void split(float2 zk, float2 znk, float2& xl, float2& xr) {
  xl = make_float2(0.5f * (zk.x + znk.x), 0.5f * (zk.y - znk.y));
  xr = make_float2(0.5f * (zk.y + znk.y), -0.5f * (zk.x - znk.x));
}

__device__ __forceinline__ double mag(float2 x) {
  return sqrt((double)x.x * x.x + (double)x.y * x.y + kMagEps);
}

template <int N>
__global__ __launch_bounds__(kBlock) void stats_kernel(int rows, int64_t T, const float* Y,
                                                       const float* tgt, double* part) {
  __shared__ float2 a[N], b[N], c[N], d[N];
  __shared__ double red[4];
  const int f = blockIdx.x, row = blockIdx.y;
  const int64_t s0 = (int64_t)f * (N / 4);
  load_frame<N>(Y + (int64_t)row * 2 * T, T, s0, a);
  load_frame<N>(tgt + (int64_t)row * 2 * T, T, s0, c);
  __syncthreads();
  lds_fft<N, false>(a, b);
  lds_fft<N, false>(c, d);
  double sd = 0.0, st = 0.0, sl = 0.0;
  for (int k = threadIdx.x; k <= N / 2; k += kBlock) {
    float2 yl, yr, tl, tr;
    split(b[k], b[(N - k) & (N - 1)], yl, yr);
    split(d[k], d[(N - k) & (N - 1)], tl, tr);
    const double my[2] = {mag(yl), mag(yr)}, mt[2] = {mag(tl), mag(tr)};
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      sd += (my[ch] - mt[ch]) * (my[ch] - mt[ch]);
      st += mt[ch] * mt[ch];
      sl += fabs(log(my[ch]) - log(mt[ch]));
    }
  }
  sd = block_sum<double>(sd, red);
  st = block_sum<double>(st, red);
  sl = block_sum<double>(sl, red);
  if (threadIdx.x == 0) {
    double* p = part + ((int64_t)f * rows + row) * 3;
    p[0] = sd;
    p[1] = st;
    p[2] = sl;
  }
}

struct Frames {
  int F[3];
  double* part[3];
};

__global__ __launch_bounds__(kBlock) void reduce_kernel(int rows, Frames fr, double* consts,
                                                        float* loss) {
  __shared__ double red[4];
  double L = 0.0;
  for (int i = 0; i < 3; ++i) {
    const int n = fr.F[i] * rows;
    double s[3] = {0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < n; q += kBlock)
      for (int j = 0; j < 3; ++j) s[j] += fr.part[i][(int64_t)q * 3 + j];
    for (int j = 0; j < 3; ++j) s[j] = block_sum<double>(s[j], red);
    if (n > 0) {
      const double nd = sqrt(s[0]), nt = sqrt(s[1]);
      const double M = (double)n * 2.0 * (kRes[i] / 2 + 1);
      L += nd / nt + s[2] / M;
      if (threadIdx.x == 0) {
        consts[2 * i] = nd > 0.0 ? 1.0 / (3.0 * nd * nt) : 0.0;
        consts[2 * i + 1] = 1.0 / (3.0 * M);
      }
    } else if (threadIdx.x == 0) {
      consts[2 * i] = consts[2 * i + 1] = 0.0;
    }
  }
  if (threadIdx.x == 0) *loss = (float)(L / 3.0);
}

template <int N>
__global__ __launch_bounds__(kBlock) void grad_kernel(int rows, int64_t T, const float* Y,
                                                      const float* tgt, const double* consts,
                                                      int res, const float* dloss, int frames,
                                                      float* fb) {
  __shared__ float2 a[N], b[N], c[N], d[N];
  const int f = blockIdx.x, row = blockIdx.y;
  const int64_t s0 = (int64_t)f * (N / 4);
  load_frame<N>(Y + (int64_t)row * 2 * T, T, s0, a);
  load_frame<N>(tgt + (int64_t)row * 2 * T, T, s0, c);
  __syncthreads();
  lds_fft<N, false>(a, b);
  lds_fft<N, false>(c, d);
  const double up = (double)*dloss;
  const double c_sc = consts[2 * res] * up, c_lm = consts[2 * res + 1] * up;
  // Hermitian spectrum of the frame gradient, both channels packed: F = F_l + i F_r (into a)
  for (int k = threadIdx.x; k <= N / 2; k += kBlock) {
    float2 x[2], t[2];
    split(b[k], b[(N - k) & (N - 1)], x[0], x[1]);
    split(d[k], d[(N - k) & (N - 1)], t[0], t[1]);
    float2 G[2];
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      const double my = mag(x[ch]), mt = mag(t[ch]);
      const double dl = log(my) - log(mt);
      const double sgn = dl > 0.0 ? 1.0 : (dl < 0.0 ? -1.0 : 0.0);
      const double gS = c_sc * (my - mt) + c_lm * sgn / my;
      G[ch] = make_float2((float)(gS * x[ch].x / my), (float)(gS * x[ch].y / my));
    }
    if (k == 0 || k == N / 2) {
      a[k] = make_float2(G[0].x, G[1].x);
    } else {
      const float2 gl = make_float2(0.5f * G[0].x, 0.5f * G[0].y);
      const float2 gr = make_float2(0.5f * G[1].x, 0.5f * G[1].y);
      a[k] = make_float2(gl.x - gr.y, gl.y + gr.x);
      a[N - k] = make_float2(gl.x + gr.y, -gl.y + gr.x);  // conj(gl) + i conj(gr)
    }
  }
  __syncthreads();
  lds_fft<N, true>(a, b);
  float* out = fb + ((int64_t)row * frames + f) * 2 * N;
  for (int n = threadIdx.x; n < N; n += kBlock) {
    const float w = hann<N>(n);
    out[n] = w * b[n].x;
    out[N + n] = w * b[n].y;
  }
}

struct FrameBufs {
  int F[3];
  const float* fb[3];
};

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

}  // namespace

size_t mrstft_ws_bytes(int rows, int64_t T) { return layout(rows, T).total; }

hipError_t launch_mrstft_loss(int rows, int64_t T, const float* Y, const float* tgt, float* loss,
                              void* ws, hipStream_t s) {
  const Layout L = layout(rows, T);
  char* base = static_cast<char*>(ws);
  Frames fr;
  for (int i = 0; i < 3; ++i) {
    fr.F[i] = frames_of(T, kRes[i]);
    fr.part[i] = reinterpret_cast<double*>(base + L.part[i]);
  }
  if (fr.F[0] > 0)
    stats_kernel<512><<<dim3(fr.F[0], rows), kBlock, 0, s>>>(rows, T, Y, tgt, fr.part[0]);
  if (fr.F[1] > 0)
    stats_kernel<1024><<<dim3(fr.F[1], rows), kBlock, 0, s>>>(rows, T, Y, tgt, fr.part[1]);
  if (fr.F[2] > 0)
    stats_kernel<2048><<<dim3(fr.F[2], rows), kBlock, 0, s>>>(rows, T, Y, tgt, fr.part[2]);
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
  if (fbs.F[0] > 0)
    grad_kernel<512><<<dim3(fbs.F[0], rows), kBlock, 0, s>>>(rows, T, Y, tgt, consts, 0, dloss,
                                                             fbs.F[0], fb0);
  if (fbs.F[1] > 0)
    grad_kernel<1024><<<dim3(fbs.F[1], rows), kBlock, 0, s>>>(rows, T, Y, tgt, consts, 1, dloss,
                                                              fbs.F[1], fb1);
  if (fbs.F[2] > 0)
    grad_kernel<2048><<<dim3(fbs.F[2], rows), kBlock, 0, s>>>(rows, T, Y, tgt, consts, 2, dloss,
                                                              fbs.F[2], fb2);
  const int64_t n = (int64_t)rows * 2 * T;
  ola_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(rows, T, fbs, dY);
  return hipGetLastError();
}

}  // namespace grafx
