// Feed-forward compressor (paper Sec. 3 "Compressor", Eqs. 8-12), parallel across nodes and
// time chunks.
//
// With equal attack and release the energy envelope g[t] = a g[t-1] + (1-a) x[t],
// x = (u_l + u_r)^2, is a linear one-pole recursion (the untruncated FIR of Eq. 9). It is computed
// exactly, in double, as a chunked scan: each block owns 2048 samples (256 threads x 8 consecutive
// samples); a thread folds its 8 samples, a Kogge-Stone scan across the wave and a fold across
// the 4 waves give every thread its incoming state. Chunks are chained in three launches: local
// chunk totals, a fixed-order carry fold per node (c_{k+1} = a^2048 c_k + total_k), then the
// final pass that rebuilds g from its carry, applies the quadratic-knee curve
// (G_u = ln(g + 1e-8); gain exp(G_y - G_u)) and writes y. Every fold has a fixed order, so the
// result does not depend on block scheduling.
//
// Adjoint (rho = sum_c ybar_c y_c, e = G_y - G_u):
//   gbar = rho de/dG_u / (g + 1e-8);  lambda[t] = gbar[t] + a lambda[t+1]  (reverse scan);
//   ubar_c = gamma ybar_c + 2 (u_l + u_r)(1 - a) lambda;
//   dL/da = sum lambda[t] (g[t-1] - x[t]);  dL/d(T, W, R) = sum rho de/d(T, W, R).
// The reverse recursion uses the same chunked scan run on reversed thread order. The forward
// carries saved by the render are the only state kept between the two calls.
#include "device_common.h"
#include "grafx_internal.h"
#include "kernels.h"

namespace grafx {
namespace {

constexpr int kPer = 8;
constexpr int kChunk = kCompChunk;  // 256 x 8
constexpr double kEps = 1e-8;

struct Coef {
  double a, b;             // alpha, 1 - alpha
  double thr, knee, c, R;  // T, W, 1/R - 1, R
  double pw[9];            // pw[d] = (a^8)^(2^d); pw[8] = a^2048
};

__device__ __forceinline__ Coef load_coef(const float* P, int slot) {
  Coef k;
  const float* p = P + (int64_t)slot * 4;
  k.a = (double)p[0];
  k.b = 1.0 - k.a;
  k.thr = (double)p[1];
  k.knee = (double)p[2];
  k.R = (double)p[3];
  k.c = 1.0 / k.R - 1.0;
  double q = k.a * k.a;
  q = q * q;
  k.pw[0] = q * q;
#pragma unroll
  for (int d = 1; d < 9; ++d) k.pw[d] = k.pw[d - 1] * k.pw[d - 1];
  return k;
}

// (a^8)^n for 0 <= n < 512
__device__ __forceinline__ double pow_a8(const Coef& k, int n) {
  double r = 1.0;
#pragma unroll
  for (int d = 0; d < 9; ++d)
    if ((n >> d) & 1) r *= k.pw[d];
  return r;
}

struct Curve {
  double e, dG, dT, dW, dR;
};

// e = G_y - G_u of the quadratic-knee curve (Eqs. 10-11) and its partial derivatives.
template <bool GRAD>
__device__ __forceinline__ Curve curve(double Gu, const Coef& k) {
  Curve o{0.0, 0.0, 0.0, 0.0, 0.0};
  const double d = Gu - k.thr;
  const bool soft = k.knee > 0.0;
  if (soft ? (Gu < k.thr - k.knee) : (Gu < k.thr)) return o;
  if (soft && Gu < k.thr + k.knee) {
    const double q = d + k.knee;
    const double w4 = 4.0 * k.knee;
    o.e = k.c * q * q / w4;
    if (GRAD) {
      o.dG = k.c * q / (2.0 * k.knee);
      o.dT = -o.dG;
      o.dW = k.c * (q / (2.0 * k.knee) - q * q / (w4 * k.knee));
      o.dR = -q * q / (w4 * k.R * k.R);
    }
    return o;
  }
  o.e = k.c * d;
  if (GRAD) {
    o.dG = k.c;
    o.dT = -k.c;
    o.dR = -d / (k.R * k.R);
  }
  return o;
}

// Chunk scan of s_out = a^8 s_in + B over the block's 256 threads (reversed thread order when
// REV). `B` is this thread's fold of its own 8 samples from a zero state; `cin` is the state
// entering the chunk. Returns the state entering this thread's samples; `chunk_out` receives the
// state leaving the chunk (every thread).
template <bool REV>
__device__ __forceinline__ double chunk_scan(double B, double cin, const Coef& k, double* wtot,
                                             double& chunk_out) {
  const int lane0 = threadIdx.x & 63, w0 = threadIdx.x >> 6;
  const int lane = REV ? 63 - lane0 : lane0;
  const int w = REV ? 3 - w0 : w0;
  double S = B;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const double o = REV ? __shfl_down(S, 1 << d, 64) : __shfl_up(S, 1 << d, 64);
    if (lane >= (1 << d)) S = fma(k.pw[d], o, S);
  }
  double ex = REV ? __shfl_down(S, 1, 64) : __shfl_up(S, 1, 64);
  if (lane == 0) ex = 0.0;
  __syncthreads();
  if (lane == 63) wtot[w] = S;
  __syncthreads();
  double P = cin, end = cin;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (v < w) P = fma(k.pw[6], P, wtot[v]);
    end = fma(k.pw[6], end, wtot[v]);
  }
  chunk_out = end;
  return fma(pow_a8(k, lane), P, ex);
}

// Stage the gather-sum of a chunk (both channels) into LDS.
__device__ __forceinline__ void stage_input(const GraphView& g, int node, int64_t t0, float* sl,
                                            float* sr) {
  const int64_t T = g.T;
  const int e0 = g.in_ptr[node], e1 = g.in_ptr[node + 1];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int idx = threadIdx.x + kBlock * q;
    const int64_t t = t0 + idx;
    float l = 0.f, r = 0.f;
    if (t < T)
      for (int e = e0; e < e1; ++e) {
        const float* row = out_row(g, g.in_src[e]);
        l += row[t];
        r += row[T + t];
      }
    sl[idx] = l;
    sr[idx] = r;
  }
}

__device__ __forceinline__ void stage_adjoint(const GraphView& g, int node, int64_t t0, float* sl,
                                              float* sr) {
  const int64_t T = g.T;
  const int o0 = g.out_ptr[node], o1 = g.out_ptr[node + 1];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int idx = threadIdx.x + kBlock * q;
    const int64_t t = t0 + idx;
    float l = 0.f, r = 0.f;
    if (t < T)
      for (int e = o0; e < o1; ++e) {
        const float* row = adj_row(g, g.out_dst[e]);
        l += row[t];
        r += row[T + t];
      }
    sl[idx] = l;
    sr[idx] = r;
  }
}

__device__ __forceinline__ double energy(const float* sl, const float* sr, int idx) {
  const double m = (double)sl[idx] + (double)sr[idx];
  return m * m;
}

__device__ __forceinline__ void store_chunk(float* row, int64_t T, int64_t t0, const float* sl,
                                            const float* sr) {
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int idx = threadIdx.x + kBlock * q;
    const int64_t t = t0 + idx;
    if (t < T) {
      row[t] = sl[idx];
      row[T + t] = sr[idx];
    }
  }
}

// ---- forward ----------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void comp_fwd_total_kernel(GraphView g, const float* P,
                                                                int node_begin, int chunks,
                                                                double* agg) {
  __shared__ float sl[kChunk], sr[kChunk];
  __shared__ double wtot[4];
  const int chunk = blockIdx.x, node = node_begin + blockIdx.y;
  const int slot = g.param_row[node];
  const Coef k = load_coef(P, slot);
  stage_input(g, node, (int64_t)chunk * kChunk, sl, sr);
  __syncthreads();
  double B = 0.0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) B = fma(k.a, B, k.b * energy(sl, sr, kPer * threadIdx.x + i));
  double end;
  chunk_scan<false>(B, 0.0, k, wtot, end);
  if (threadIdx.x == 0) agg[(int64_t)slot * chunks + chunk] = end;
}

// carry[k] = state entering chunk k; carry[0] = 0 (g[-1] = 0), carry[k+1] = a^2048 carry[k] +
// agg[k]. One thread per node walks its chunks in order.
__global__ __launch_bounds__(64) void comp_carry_kernel(const int32_t* param_row, const float* P,
                                                        int node_begin, int chunks,
                                                        const double* agg, double* carry) {
  if (threadIdx.x != 0) return;
  const int slot = param_row[node_begin + blockIdx.x];
  const Coef k = load_coef(P, slot);
  const double A = k.pw[8];
  const double* a = agg + (int64_t)slot * chunks;
  double* c = carry + (int64_t)slot * chunks;
  double s = 0.0;
  for (int i = 0; i < chunks; ++i) {
    c[i] = s;
    s = fma(A, s, a[i]);
  }
}

__global__ __launch_bounds__(kBlock) void comp_fwd_apply_kernel(GraphView g, float* U,
                                                                const float* P, int node_begin,
                                                                int chunks, const double* carry) {
  __shared__ float sl[kChunk], sr[kChunk];
  __shared__ double wtot[4];
  const int chunk = blockIdx.x, node = node_begin + blockIdx.y;
  const int slot = g.param_row[node];
  const Coef k = load_coef(P, slot);
  const int64_t t0 = (int64_t)chunk * kChunk;
  stage_input(g, node, t0, sl, sr);
  __syncthreads();
  const int i0 = kPer * threadIdx.x;
  double B = 0.0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) B = fma(k.a, B, k.b * energy(sl, sr, i0 + i));
  double end;
  double s = chunk_scan<false>(B, carry[(int64_t)slot * chunks + chunk], k, wtot, end);
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    s = fma(k.a, s, k.b * energy(sl, sr, i0 + i));
    const Curve cv = curve<false>(log(s + kEps), k);
    const double gam = exp(cv.e);
    sl[i0 + i] = (float)(gam * (double)sl[i0 + i]);
    sr[i0 + i] = (float)(gam * (double)sr[i0 + i]);
  }
  __syncthreads();
  store_chunk(U + (int64_t)node * 2 * g.T, g.T, t0, sl, sr);
}

// ---- adjoint ----------------------------------------------------------------------------------

// Per-sample adjoint quantities of one thread's 8 samples.
struct Local {
  double gv[kPer];    // envelope g
  double gbar[kPer];  // dL/dg (direct part, before the recursion)
  float gam[kPer];    // gain
  double E;           // envelope entering the thread's first sample
  double accT, accW, accR;
};

__device__ __forceinline__ void adjoint_local(const float* ul, const float* ur, const float* yl,
                                              const float* yr, const Coef& k, double cin,
                                              double* wtot, Local& L) {
  const int i0 = kPer * threadIdx.x;
  double B = 0.0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) B = fma(k.a, B, k.b * energy(ul, ur, i0 + i));
  double end;
  L.E = chunk_scan<false>(B, cin, k, wtot, end);
  double s = L.E;
  L.accT = L.accW = L.accR = 0.0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    s = fma(k.a, s, k.b * energy(ul, ur, i0 + i));
    L.gv[i] = s;
    const Curve cv = curve<true>(log(s + kEps), k);
    const double gam = exp(cv.e);
    const double rho = gam * ((double)yl[i0 + i] * (double)ul[i0 + i] +
                              (double)yr[i0 + i] * (double)ur[i0 + i]);
    L.gam[i] = (float)gam;
    L.gbar[i] = rho * cv.dG / (s + kEps);
    L.accT += rho * cv.dT;
    L.accW += rho * cv.dW;
    L.accR += rho * cv.dR;
  }
}

__global__ __launch_bounds__(kBlock) void comp_bwd_total_kernel(GraphView g, const float* P,
                                                                int node_begin, int chunks,
                                                                const double* carry,
                                                                double* ragg) {
  __shared__ float ul[kChunk], ur[kChunk], yl[kChunk], yr[kChunk];
  __shared__ double wtot[4];
  const int chunk = blockIdx.x, node = node_begin + blockIdx.y;
  const int slot = g.param_row[node];
  const Coef k = load_coef(P, slot);
  const int64_t t0 = (int64_t)chunk * kChunk;
  stage_input(g, node, t0, ul, ur);
  stage_adjoint(g, node, t0, yl, yr);
  __syncthreads();
  Local L;
  adjoint_local(ul, ur, yl, yr, k, carry[(int64_t)slot * chunks + chunk], wtot, L);
  double R = 0.0;
#pragma unroll
  for (int i = kPer - 1; i >= 0; --i) R = fma(k.a, R, L.gbar[i]);
  double end;
  chunk_scan<true>(R, 0.0, k, wtot, end);
  if (threadIdx.x == 0) ragg[(int64_t)slot * chunks + chunk] = end;
}

// rcarry[k] = lambda entering chunk k from the right (lambda at the first sample after it):
// rcarry[last] = 0, rcarry[k-1] = ragg[k] + a^2048 rcarry[k].
__global__ __launch_bounds__(64) void comp_rcarry_kernel(const int32_t* param_row, const float* P,
                                                         int node_begin, int chunks,
                                                         const double* ragg, double* rcarry) {
  if (threadIdx.x != 0) return;
  const int slot = param_row[node_begin + blockIdx.x];
  const Coef k = load_coef(P, slot);
  const double A = k.pw[8];
  const double* a = ragg + (int64_t)slot * chunks;
  double* c = rcarry + (int64_t)slot * chunks;
  double s = 0.0;
  for (int i = chunks - 1; i >= 0; --i) {
    c[i] = s;
    s = fma(A, s, a[i]);
  }
}

__global__ __launch_bounds__(kBlock) void comp_bwd_apply_kernel(GraphView g, float* dU,
                                                                const float* P, int node_begin,
                                                                int chunks, const double* carry,
                                                                const double* rcarry,
                                                                double* part) {
  __shared__ float ul[kChunk], ur[kChunk], yl[kChunk], yr[kChunk];
  __shared__ double wtot[4];
  __shared__ double red[4];
  const int chunk = blockIdx.x, node = node_begin + blockIdx.y;
  const int slot = g.param_row[node];
  const Coef k = load_coef(P, slot);
  const int64_t t0 = (int64_t)chunk * kChunk;
  stage_input(g, node, t0, ul, ur);
  stage_adjoint(g, node, t0, yl, yr);
  __syncthreads();
  Local L;
  adjoint_local(ul, ur, yl, yr, k, carry[(int64_t)slot * chunks + chunk], wtot, L);
  double R = 0.0;
#pragma unroll
  for (int i = kPer - 1; i >= 0; --i) R = fma(k.a, R, L.gbar[i]);
  double end;
  double lam = chunk_scan<true>(R, rcarry[(int64_t)slot * chunks + chunk], k, wtot, end);
  const int i0 = kPer * threadIdx.x;
  double accA = 0.0;
#pragma unroll
  for (int i = kPer - 1; i >= 0; --i) {
    lam = fma(k.a, lam, L.gbar[i]);
    const double x = energy(ul, ur, i0 + i);
    const double gprev = i > 0 ? L.gv[i - 1] : L.E;
    accA += lam * (gprev - x);
    const double mid = 2.0 * ((double)ul[i0 + i] + (double)ur[i0 + i]) * k.b * lam;
    yl[i0 + i] = (float)((double)L.gam[i] * (double)yl[i0 + i] + mid);
    yr[i0 + i] = (float)((double)L.gam[i] * (double)yr[i0 + i] + mid);
  }
  const double sA = block_sum<double>(accA, red);
  const double sT = block_sum<double>(L.accT, red);
  const double sW = block_sum<double>(L.accW, red);
  const double sR = block_sum<double>(L.accR, red);
  if (threadIdx.x == 0) {
    double* p = part + ((int64_t)slot * chunks + chunk) * 4;
    p[0] = sA;
    p[1] = sT;
    p[2] = sW;
    p[3] = sR;
  }
  store_chunk(dU + (int64_t)node * 2 * g.T, g.T, t0, yl, yr);
}

}  // namespace

int comp_chunks(int64_t T) { return (int)((T + kChunk - 1) / kChunk); }

hipError_t launch_comp_fwd(const GraphView& g, float* U, const float* P, int node_begin,
                           int n_nodes, double* agg, double* carry, hipStream_t s) {
  const int chunks = comp_chunks(g.T);
  const dim3 grid((unsigned)chunks, (unsigned)n_nodes);
  comp_fwd_total_kernel<<<grid, kBlock, 0, s>>>(g, P, node_begin, chunks, agg);
  comp_carry_kernel<<<n_nodes, 64, 0, s>>>(g.param_row, P, node_begin, chunks, agg, carry);
  comp_fwd_apply_kernel<<<grid, kBlock, 0, s>>>(g, U, P, node_begin, chunks, carry);
  return hipGetLastError();
}

hipError_t launch_comp_bwd(const GraphView& g, float* dU, const float* P, int node_begin,
                           int n_nodes, const double* carry, double* ragg, double* rcarry,
                           double* part, hipStream_t s) {
  const int chunks = comp_chunks(g.T);
  const dim3 grid((unsigned)chunks, (unsigned)n_nodes);
  comp_bwd_total_kernel<<<grid, kBlock, 0, s>>>(g, P, node_begin, chunks, carry, ragg);
  comp_rcarry_kernel<<<n_nodes, 64, 0, s>>>(g.param_row, P, node_begin, chunks, ragg, rcarry);
  comp_bwd_apply_kernel<<<grid, kBlock, 0, s>>>(g, dU, P, node_begin, chunks, carry, rcarry,
                                                part);
  return hipGetLastError();
}

}  // namespace grafx
