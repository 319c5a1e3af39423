// Multitap delay (paper Sec. 3 "Multitap delay", Eq. 14) with M 100 ms slots per channel:
// y_c[t] = sum_m sum_{j=-19}^{19} c_{c,m}[j] u_c[t - d_{c,m} - j]. Two node types share these
// kernels, templated on M: the 2 s delay of the paper (M = 20, 880 parameters) and a 500 ms one
// (M = 5, 220 parameters).
//
// Design (once per render): the integer delay of slot m is (m * 4410) plus
// rint(-arg(z) * 4410 / 2 pi) mod 4410, decided in float32; each slot's 39-tap zero-phase FIR is
// built from its 20 log-magnitudes like the EQ (N = 39, symmetric Hann), in double.
// Filtering: one block per 2048 outputs of one node; for each (channel, slot) the 2086-sample
// input window is staged in LDS and every thread forms 8 consecutive outputs from registers.
// Adjoint: the input adjoint is the correlation with the same taps (a separate launch), and the
// tap gradient c-bar_{c,m}[j] = sum_t ybar_c[t] u_c[t - d - j] is accumulated per block over a
// fixed group of tiles, reduced in a fixed order and mapped back to the log-magnitudes through
// the design. By default the delay times are not differentiated (their phasor gradients are 0).
//
// Delay-time surrogate (Sec. 3 "Multitap delay", Eq. 15), an option of the schedule: the phasor z
// of slot m gets the straight-through gradient of the surrogate impulse
// s[n] = Re (1/N) sum_{k<N} z^k e^(2 pi i k n / N) (N = 4410 lags from the slot's start), which is
// the unit impulse at the slot's integer delay when z lies on the unit circle at that delay. With
// G[n] = dL/ds[n] = sum_j c[j] R[4410 m + n + j - 19] (R[l] = sum_t ybar[t] u[t - l], the
// cross-correlation of the output adjoint and the input, from the partitioned correlation of the
// reverb's FIR gradient with the output adjoint delayed by 19 samples so that lags start at -19),
// dL/dRe z = Re Q and dL/dIm z = -Im Q with Q = sum_n G[n] s'(z)[n]
// = (1/N) sum_{k>=1} k z^(k-1) sum_n G[n] e^(2 pi i k n / N), all in double.
#include <type_traits>

#include "device_common.h"
#include "grafx_internal.h"
#include "kernels.h"

namespace grafx {
namespace {

constexpr int kHop = 2048;
constexpr int kHalf = 19;                 // taps j = -19..19
constexpr int kWin = kHop + 2 * kHalf;    // 2086
constexpr int kPer = kHop / kBlock;       // 8 outputs per thread
template <int M>
__global__ __launch_bounds__(kBlock) void delay_design_kernel(const float* P, float* taps,
                                                              int32_t* offs) {
  constexpr int kRow = delay_row(M), kCoef = delay_coef(M);
  const int node = blockIdx.x;
  const float* p = P + (int64_t)node * kRow;
  for (int i = threadIdx.x; i < kCoef; i += kBlock) {
    const int cm = i / kDelayFir, j = i % kDelayFir - kHalf;  // cm = c * 5 + m
    const float* q = p + cm * 22;
    double acc = exp((double)q[2]);
    for (int k = 1; k <= kHalf; ++k) acc += 2.0 * exp((double)q[2 + k]) * cospi(2.0 * k * j / 39.0);
    const double h0 = acc / 39.0;
    const double win = 0.5 + 0.5 * cospi((double)j / kHalf);
    taps[(int64_t)node * kCoef + i] = (float)(win * h0);
  }
  if (threadIdx.x < 2 * M) {
    const int cm = threadIdx.x, m = cm % M;
    const float* q = p + cm * 22;
    const float kScale = (float)(4410.0 / (2.0 * 3.14159265358979323846));
    const float ph = atan2f(q[1], q[0]);
    const int r = (int)rintf(-ph * kScale);
    const int d = ((r % kDelaySlot) + kDelaySlot) % kDelaySlot;
    offs[(int64_t)node * 2 * M + cm] = m * kDelaySlot + d;
  }
}

// Stage x[base .. base + len) (len <= kWin) of one channel of a node's gather-sum (in: input
// edges over U/S, adj: output edges over dU/dY) into LDS. Each row is read through a buffer
// resource sized to its node's length, so samples before 0 or past the length read as zero
// without a branch, and all of a row's loads are issued before any is consumed.
template <bool ADJ>
__device__ __forceinline__ void stage_window(const GraphView& g, int node, int c, int64_t base,
                                             int len, float* w) {
  constexpr int kQ = (kWin + kBlock - 1) / kBlock;
  const int64_t T = g.T;
  const int e0 = ADJ ? g.out_ptr[node] : g.in_ptr[node];
  const int e1 = ADJ ? g.out_ptr[node + 1] : g.in_ptr[node + 1];
  const int t_first = (int)base + (int)threadIdx.x;  // base > -2^30: negative offsets read 0
  float s[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) s[q] = 0.f;
  for (int e = e0; e < e1; ++e) {
    const int other = ADJ ? g.out_dst[e] : g.in_src[e];
    const float* row = (ADJ ? adj_row(g, other) : out_row(g, other)) + (int64_t)c * T;
    const auto rs = row_rsrc(row, node_len(g, other));
    float x[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) x[q] = bload(rs, t_first + kBlock * q);
#pragma unroll
    for (int q = 0; q < kQ; ++q) s[q] += x[q];
  }
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int idx = (int)threadIdx.x + kBlock * q;
    if (idx < len) w[idx] = s[q];
  }
}

// out[o] += sum_{j} c[j] w[o + 19 - j] (forward: convolution; window starts at t0 - d - 19) or
// out[o] += sum_{j} c[j] w[o + 19 + j] (adjoint: correlation; window starts at t0 + d - 19).
template <bool ADJ>
__device__ __forceinline__ void apply_taps(const float* w, const float* c, float* acc) {
  const int o0 = kPer * threadIdx.x;
  float x[kPer + 2 * kHalf];
#pragma unroll
  for (int i = 0; i < kPer + 2 * kHalf; ++i) x[i] = w[o0 + i];
#pragma unroll
  for (int jj = 0; jj < kDelayFir; ++jj) {
    const float cj = c[jj];  // tap j = jj - 19
#pragma unroll
    for (int i = 0; i < kPer; ++i) acc[i] += cj * x[ADJ ? i + jj : i + 2 * kHalf - jj];
  }
}

template <bool ADJ, int M>
__global__ __launch_bounds__(kBlock) void delay_conv_kernel(GraphView g, float* out,
                                                            const float* taps,
                                                            const int32_t* offs, int node_begin,
                                                            int tiles) {
  __shared__ float w[kWin];
  __shared__ float ys[2][kHop];
  const int tile = blockIdx.x, node = node_begin + blockIdx.y;
  const int slot = g.param_row[node];
  const int64_t T = g.T, t0 = (int64_t)tile * kHop, Tn = node_len(g, node);
  if (t0 >= Tn) return;  // tile past the node's length (uniform over the block)
  const float* cn = taps + (int64_t)slot * delay_coef(M);
  for (int c = 0; c < 2; ++c) {
    float acc[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) acc[i] = 0.f;
    for (int m = 0; m < M; ++m) {
      const int d = offs[(int64_t)slot * 2 * M + c * M + m];
      const int64_t base = ADJ ? t0 + d - kHalf : t0 - d - kHalf;
      __syncthreads();
      stage_window<ADJ>(g, node, c, base, kWin, w);
      __syncthreads();
      apply_taps<ADJ>(w, cn + (c * M + m) * kDelayFir, acc);
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) ys[c][kPer * threadIdx.x + i] = acc[i];
  }
  __syncthreads();
  float* y = out + (int64_t)node * 2 * T;
  for (int idx = threadIdx.x; idx < kHop; idx += kBlock) {
    const int64_t t = t0 + idx;
    if (t < Tn) {
      store_nt(y + t, ys[0][idx]);
      store_nt(y + T + t, ys[1][idx]);
    }
  }
  (void)tiles;
}

// Tiles per tap-gradient block: a setting of the schedule (4, 8 or 16; 16 by default), not a
// function of T, so a node's partial sums are grouped the same way whatever the row stride (a
// graph merged with longer ones gets the same bits as alone). More tiles amortise the block
// reduction of the 39 sums per channel-tap; fewer give short steps more blocks.

// Tap gradients: part[slot][group][c*M+m][j] = sum over the group's tiles of
// sum_t ybar_c[t] u_c[t - d - j]. One block per (node, group, channel-slot): the ten sums of a
// group are independent, so splitting them over blocks keeps ten times more stage-and-compute
// chains in flight (the kernel is bound by their latency). Logical blocks are laid out node,
// group, channel-slot and spread XCD-contiguously, so the five slots of a channel, which stage
// the same adjoint tiles, share an L2.
template <int M>
__global__ __launch_bounds__(kBlock) void delay_tapgrad_kernel(GraphView g, const int32_t* offs,
                                                               int node_begin, int tiles,
                                                               int groups, float* part) {
  __shared__ float w[kWin];
  __shared__ float yb[kHop];
  __shared__ float red[4][kDelayFir];
  constexpr int kCM = 2 * M;
  const int nb = (int)(gridDim.x * gridDim.y);
  const int lb = xcd_logical_block((int)(blockIdx.y * gridDim.x + blockIdx.x), nb);
  const int per_node = groups * kCM;
  const int node = node_begin + lb / per_node;
  const int group = (lb % per_node) / kCM, cm = lb % kCM;
  const int slot = g.param_row[node];
  const int tiles_n = (int)((node_len(g, node) + kHop - 1) / kHop);  // the node's own tiles
  const int tile_end = min(min(tiles, tiles_n), (group + 1) * g.tap_tiles);
  const int o0 = kPer * threadIdx.x;
  {
    const int c = cm / M;
    const int d = offs[(int64_t)slot * 2 * M + cm];
    float acc[kDelayFir];
#pragma unroll
    for (int jj = 0; jj < kDelayFir; ++jj) acc[jj] = 0.f;
    for (int tile = group * g.tap_tiles; tile < tile_end; ++tile) {
      const int64_t t0 = (int64_t)tile * kHop;
      __syncthreads();
      stage_window<false>(g, node, c, t0 - d - kHalf, kWin, w);
      stage_window<true>(g, node, c, t0, kHop, yb);
      __syncthreads();
      float x[kPer + 2 * kHalf];
#pragma unroll
      for (int q = 0; q < kPer + 2 * kHalf; ++q) x[q] = w[o0 + q];
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const float yv = yb[o0 + q];
#pragma unroll
        for (int jj = 0; jj < kDelayFir; ++jj) acc[jj] += yv * x[q + 2 * kHalf - jj];
      }
    }
    // block reduction of the 39 partial sums (fixed order)
#pragma unroll
    for (int jj = 0; jj < kDelayFir; ++jj) acc[jj] = wave_sum(acc[jj]);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
      for (int jj = 0; jj < kDelayFir; ++jj) red[threadIdx.x >> 6][jj] = acc[jj];
    __syncthreads();
    if (threadIdx.x < kDelayFir) {
      const int jj = threadIdx.x;
      part[(((int64_t)slot * groups + group) * 2 * M + cm) * kDelayFir + jj] =
          red[0][jj] + red[1][jj] + red[2][jj] + red[3][jj];
    }
  }
}

// Sum tap-gradient partials over groups and map them to the log-magnitudes:
// dL/dlogmag_k = A_k (kappa_k / 39) sum_j cbar[j] v[j] cos(2 pi k j / 39).
template <int M>
__global__ __launch_bounds__(kBlock) void delay_grad_kernel(const float* P, const float* part,
                                                            int groups, float* dP) {
  constexpr int kRow = delay_row(M), kCoef = delay_coef(M);
  __shared__ double cb[kCoef];
  const int slot = blockIdx.x;
  for (int i = threadIdx.x; i < kCoef; i += kBlock) {
    double s = 0.0;
    for (int gi = 0; gi < groups; ++gi) s += part[((int64_t)slot * groups + gi) * kCoef + i];
    const int j = i % kDelayFir - kHalf;
    cb[i] = s * (0.5 + 0.5 * cospi((double)j / kHalf));
  }
  __syncthreads();
  const float* p = P + (int64_t)slot * kRow;
  float* d = dP + (int64_t)slot * kRow;
  for (int i = threadIdx.x; i < kRow; i += kBlock) {
    const int cm = i / 22, q = i % 22;
    if (q < 2) {
      d[i] = 0.f;
      continue;
    }
    const int k = q - 2;
    double acc = 0.0;
    for (int jj = 0; jj < kDelayFir; ++jj) acc += cb[cm * kDelayFir + jj] * cospi(2.0 * k * (jj - kHalf) / 39.0);
    const double kappa = k == 0 ? 1.0 : 2.0;
    d[i] = (float)(exp((double)p[i]) * kappa / 39.0 * acc);
  }
}

// Straight-through phasor gradient of one (node slot, channel x slot) pair: G into LDS, then Q as
// above, each thread taking the k = 1 + thread, 1 + thread + 256, ... terms; the inner sum over n
// steps the phasor e^(2 pi i k n / N) by multiplication, restarting from an exact value every 256
// steps; per-thread partials are added in a fixed order.
template <int M>
__global__ __launch_bounds__(kBlock) void delay_phasor_grad_kernel(const float* P,
                                                                   const float* taps,
                                                                   const float* R, int64_t Lr,
                                                                   float* dP) {
  constexpr int kRow = delay_row(M);
  __shared__ double G[kDelaySlot];
  __shared__ double2 red[kBlock / 64];
  const int slot = blockIdx.x, cm = blockIdx.y;  // cm = channel * M + slot
  const int c = cm / M, m = cm % M;
  const float* tp = taps + (int64_t)slot * delay_coef(M) + cm * kDelayFir;
  const float* Rc = R + ((int64_t)slot * 2 + c) * Lr + (int64_t)m * kDelaySlot;
  for (int n = threadIdx.x; n < kDelaySlot; n += kBlock) {
    double acc = 0.0;
    for (int j = 0; j < kDelayFir; ++j) acc = fma((double)tp[j], (double)Rc[n + j], acc);
    G[n] = acc;
  }
  __syncthreads();
  const float* q = P + (int64_t)slot * kRow + cm * 22;
  const double zr = q[0], zi = q[1];
  const double lr = 0.5 * log(zr * zr + zi * zi), th = atan2(zi, zr);  // principal log z
  double qr = 0.0, qi = 0.0;
  for (int k = 1 + threadIdx.x; k < kDelaySlot; k += kBlock) {
    double gr = 0.0, gi = 0.0, sr, si;  // the step e^(2 pi i k / N)
    sincospi(2.0 * (double)k / kDelaySlot, &si, &sr);
    for (int n0 = 0; n0 < kDelaySlot; n0 += 256) {
      double wr, wi;  // e^(2 pi i k n0 / N), exactly
      sincospi(2.0 * (double)(((int64_t)k * n0) % kDelaySlot) / kDelaySlot, &wi, &wr);
      const int n1 = min(n0 + 256, kDelaySlot);
      for (int n = n0; n < n1; ++n) {
        gr = fma(G[n], wr, gr);
        gi = fma(G[n], wi, gi);
        const double t = wr * sr - wi * si;
        wi = fma(wr, si, wi * sr);
        wr = t;
      }
    }
    // k z^(k - 1) = k exp((k - 1) log z)
    double sn, cs;
    sincos((double)(k - 1) * th, &sn, &cs);
    const double mag = (double)k * exp((double)(k - 1) * lr);
    const double ar = mag * cs, ai = mag * sn;
    qr += ar * gr - ai * gi;
    qi += ar * gi + ai * gr;
  }
  qr = wave_sum(qr);
  qi = wave_sum(qi);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double2(qr, qi);
  __syncthreads();
  if (threadIdx.x == 0) {
    double sr = 0.0, si = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      sr += red[w].x;
      si += red[w].y;
    }
    float* d = dP + (int64_t)slot * kRow + cm * 22;
    d[0] = (float)(sr / kDelaySlot);
    d[1] = (float)(-si / kDelaySlot);
  }
}

// Optimiser-side treatment of the phasor gradients (the paper normalises each delay's gradient and
// pulls z towards the unit circle, without constants): every (re z, im z) gradient pair is scaled
// to unit length (a zero pair stays zero), then the gradient of weight * (|z| - 1)^2,
// 2 weight (|z| - 1) z / |z| (zero at z = 0), is added. One thread per phasor.
__global__ __launch_bounds__(kBlock) void delay_phasor_regularise_kernel(int M, int n,
                                                                         const float* P, float* dP,
                                                                         float weight) {
  const int i = blockIdx.x * kBlock + threadIdx.x;  // phasor index: node * 2 M + c * M + m
  if (i >= n * 2 * M) return;
  const int64_t o = (int64_t)i * 22;  // rows are [channel][slot][22], contiguous per node
  const double gr = dP[o], gi = dP[o + 1];
  const double gn = sqrt(gr * gr + gi * gi);
  const double zr = P[o], zi = P[o + 1];
  const double r = sqrt(zr * zr + zi * zi);
  const double s = r > 0.0 ? 2.0 * (double)weight * (r - 1.0) / r : 0.0;
  dP[o] = (float)((gn > 0.0 ? gr / gn : 0.0) + s * zr);
  dP[o + 1] = (float)((gn > 0.0 ? gi / gn : 0.0) + s * zi);
}

}  // namespace

int delay_tiles(int64_t T) { return (int)((T + kHop - 1) / kHop); }

int delay_groups(int64_t T, int tap_tiles) {
  return (delay_tiles(T) + tap_tiles - 1) / tap_tiles;
}

// Calls body(std::integral_constant<int, M>) for the slot counts the library supports.
template <typename F>
hipError_t with_slots(int M, F&& body) {
  if (M == kDelayTaps) return body(std::integral_constant<int, kDelayTaps>{});
  if (M == kDelayTapsLong) return body(std::integral_constant<int, kDelayTapsLong>{});
  return hipErrorInvalidValue;
}

hipError_t launch_delay_design(int M, const float* P, int n, float* taps, int32_t* offs,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  return with_slots(M, [&](auto m) {
    delay_design_kernel<decltype(m)::value><<<n, kBlock, 0, s>>>(P, taps, offs);
    return hipGetLastError();
  });
}

hipError_t launch_delay_fwd(int M, const GraphView& g, float* U, const float* taps,
                            const int32_t* offs, int node_begin, int n_nodes, hipStream_t s) {
  const int tiles = delay_tiles(g.T);
  return with_slots(M, [&](auto m) {
    delay_conv_kernel<false, decltype(m)::value><<<dim3(tiles, n_nodes), kBlock, 0, s>>>(
        g, U, taps, offs, node_begin, tiles);
    return hipGetLastError();
  });
}

hipError_t launch_delay_bwd(int M, const GraphView& g, float* dU, const float* taps,
                            const int32_t* offs, int node_begin, int n_nodes, float* part,
                            hipStream_t s) {
  const int tiles = delay_tiles(g.T);
  const int groups = delay_groups(g.T, g.tap_tiles);
  return with_slots(M, [&](auto m) {
    constexpr int kM = decltype(m)::value;
    delay_conv_kernel<true, kM><<<dim3(tiles, n_nodes), kBlock, 0, s>>>(g, dU, taps, offs,
                                                                        node_begin, tiles);
    delay_tapgrad_kernel<kM><<<dim3(groups * 2 * kM, n_nodes), kBlock, 0, s>>>(
        g, offs, node_begin, tiles, groups, part);
    return hipGetLastError();
  });
}

hipError_t launch_delay_grad(int M, const float* P, const float* part, int n, int groups,
                             float* dP, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  return with_slots(M, [&](auto m) {
    delay_grad_kernel<decltype(m)::value><<<n, kBlock, 0, s>>>(P, part, groups, dP);
    return hipGetLastError();
  });
}

hipError_t launch_delay_phasor_regularise(int M, int n, const float* P, float* dP, float weight,
                                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int phasors = n * 2 * M;
  delay_phasor_regularise_kernel<<<(phasors + kBlock - 1) / kBlock, kBlock, 0, s>>>(M, n, P, dP,
                                                                                   weight);
  return hipGetLastError();
}

hipError_t launch_delay_phasor_grad(int M, const float* P, const float* taps, const float* R,
                                    int n, float* dP, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  return with_slots(M, [&](auto m) {
    constexpr int kM = decltype(m)::value;
    delay_phasor_grad_kernel<kM><<<dim3(n, 2 * kM), kBlock, 0, s>>>(P, taps, R,
                                                                    delay_sur_len(kM), dP);
    return hipGetLastError();
  });
}

}  // namespace grafx
