// Feed-forward compressor (paper Sec. 3 "Compressor", Eqs. 8-12) and noisegate (Sec. 3
// "Noisegate": the same envelope with a downward-expander curve), parallel across nodes and
// time chunks, one pass over the signal per direction.
//
// With equal attack and release the energy envelope g[t] = a g[t-1] + (1-a) x[t],
// x = (u_l + u_r)^2, is a linear one-pole recursion (the untruncated FIR of Eq. 9). It is computed
// in double as a chunked scan: a block owns a chunk of 3072 samples (256 threads x 12 consecutive
// samples); a thread folds its samples, a Kogge-Stone scan across the wave and a fold across the
// 4 waves give every thread its state relative to the chunk start. The chunk then publishes its
// total (the state it would leave from a zero start) and folds the totals of all earlier chunks
// of its node, c_k = sum_{j<k} total_j A^(k-1-j), A = a^3072, as one block-wide sum in a fixed
// order. Folding totals (never partially folded prefixes) keeps the arithmetic independent of
// timing, so results are deterministic and do not depend on the schedule. A block lives through
// several dependent memory round trips (ticket, loads, publish and wait, stores); the chunk size
// is chosen so that a 17-node step of 2^18 samples is resident in one round of blocks (24 KB of
// LDS and at most 80 VGPRs per thread give 6 blocks per CU), since a second round costs a whole
// block lifetime.
//
// A block's node comes from its block id; its chunk within the node comes from an atomic ticket
// on that node's counter (one cache line per counter), taken when the block starts, so every
// chunk a block waits for belongs to a block that started earlier and publishes without waiting:
// the waits always end. A total is published as one 64-bit atomic store at device scope over a
// "not ready" sentinel and read back by 64-bit atomic loads at device scope (the XCDs do not
// share an L2; device-scope atomics bypass the non-coherent caches). The reader consumes only
// that word, so no ordering with other data is needed: the accesses are relaxed, which avoids L2
// write-back and invalidation. Every wait is bounded; a wait that runs out records an error word
// and poisons its result instead of spinning forever.
//
// The gain curve G_u = ln(g + 1e-8), quadratic knee, gain exp(G_y - G_u) is evaluated in float.
//
// Adjoint (rho = sum_c ybar_c y_c, e = G_y - G_u):
//   gbar = rho de/dG_u / (g + 1e-8);  lambda[t] = gbar[t] + a lambda[t+1]  (reverse scan);
//   ubar_c = gamma ybar_c + 2 (u_l + u_r)(1 - a) lambda;
//   dL/da = sum lambda[t] (g[t-1] - x[t]);  dL/d(T, W, R) = sum rho de/d(T, W, R).
// The adjoint takes chunks from the end of each node backwards and runs the same scan on
// reversed thread order; the envelope entering each chunk is kept from the forward call.
#include "device_common.h"
#include "dynamics.h"
#include "grafx_internal.h"
#include "kernels.h"

namespace grafx {
namespace {

using namespace dyn;


struct Coef {
  double a, b;        // alpha, 1 - alpha
  float thr, knee;    // T, W
  float c;            // 1/R - 1 (compressor)
  float g1;           // 1 - R (noisegate)
  float inv2w, inv4w; // 1/(2W), 1/(4W)
  float invR2;        // 1/R^2
  double pw[9];       // pw[d] = (a^kPer)^(2^d); pw[8] = a^kChunk
  double logA;        // ln(a^kChunk), -inf for a = 0
};

__device__ __forceinline__ Coef load_coef(const float* P, int slot) {
  Coef k;
  const float* p = P + (int64_t)slot * 4;
  k.a = (double)p[0];
  k.b = 1.0 - k.a;
  k.thr = p[1];
  k.knee = p[2];
  const float R = p[3];
  k.c = 1.0f / R - 1.0f;
  k.g1 = 1.0f - R;
  k.inv2w = k.knee > 0.f ? 1.0f / (2.f * k.knee) : 0.f;
  k.inv4w = k.knee > 0.f ? 1.0f / (4.f * k.knee) : 0.f;
  k.invR2 = 1.0f / (R * R);
  k.logA = (double)kChunk * log(fabs(k.a));  // a^kChunk = |a|^kChunk: kChunk is even
  double q = 1.0, b = k.a;  // a^kPer by binary powering
  for (int e = kPer; e > 0; e >>= 1) {
    if (e & 1) q *= b;
    b *= b;
  }
  k.pw[0] = q;
#pragma unroll
  for (int d = 1; d < 9; ++d) k.pw[d] = k.pw[d - 1] * k.pw[d - 1];
  return k;
}

// (a^kPer)^n for 0 <= n < 512
__device__ __forceinline__ double pow_a8(const Coef& k, int n) {
  double r = 1.0;
#pragma unroll
  for (int d = 0; d < 9; ++d)
    if ((n >> d) & 1) r *= k.pw[d];
  return r;
}

template <bool GRAD, bool GATE>
__device__ __forceinline__ Curve curve(float Gu, const Coef& k) {
  if constexpr (GATE) return gate_curve<GRAD>(Gu, k);
  else return comp_curve<GRAD>(Gu, k);
}

// Chunk scan of s_out = a^kPer s_in + B over the block's 256 threads (reversed thread order when
// REV), from a zero state entering the chunk. Returns the state entering this thread's samples;
// `total` receives the state leaving the chunk (every thread). Thread J's state for a non-zero
// entering state c is the returned value plus (a^kPer)^J' c, J' = J (forward) or 255 - J (REV).
template <bool REV>
__device__ __forceinline__ double chunk_scan(double B, const Coef& k, double* wtot, double& total) {
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
  double P = 0.0, end = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (v < w) P = fma(k.pw[6], P, wtot[v]);
    end = fma(k.pw[6], end, wtot[v]);
  }
  total = end;
  return fma(pow_a8(k, lane), P, ex);
}


__device__ __forceinline__ int scan_index(bool rev) {
  return rev ? kBlock - 1 - (int)threadIdx.x : (int)threadIdx.x;
}

// Entering state of chunk k: fixed-order block-wide sum over the published totals of the
// chunks before it (REV: after it), weighted by A^(distance - 1). The adjacent chunk's weight is
// exactly 1, so a = 0 (A = 0, logA = -inf) gives the plain recursion's carry without 0 * inf.
__device__ __forceinline__ double carry_weight(int dist, const Coef& c) {
  return dist == 0 ? 1.0 : exp((double)dist * c.logA);
}

template <bool REV>
__device__ __forceinline__ double chunk_carry(uint64_t* tot, int k, int chunks, const Coef& c,
                                              unsigned* err, int polls, double* red) {
  double s = 0.0;
  if (!REV) {
    for (int j = threadIdx.x; j < k; j += kBlock)
      s += await_total(tot + j, err, polls) * carry_weight(k - 1 - j, c);
  } else {
    for (int j = k + 1 + threadIdx.x; j < chunks; j += kBlock)
      s += await_total(tot + j, err, polls) * carry_weight(j - k - 1, c);
  }
  return block_sum<double>(s, red);
}

// ---- forward ----------------------------------------------------------------------------------

template <bool RAGGED, bool GATE>
__global__ __launch_bounds__(kBlock) void comp_fwd_kernel(GraphView g, float* U, const float* P,
                                                          int node_begin, int n_nodes, int chunks,
                                                          int ws_off, uint64_t* agg, double* carry,
                                                          unsigned* ticket, unsigned* err) {
  __shared__ float sl[kLdsChunk], sr[kLdsChunk];
  __shared__ double wtot[4], red[4];
  __shared__ int sh_ticket;
  const int node = node_begin + block_node(g, n_nodes, chunks);
  const int slot = g.param_row[node];  // row in P
  const int ws = slot + ws_off;         // row of the dynamics workspace (compressors, then gates)
  const int chunk = take_ticket(ticket + (int64_t)ws * kCompTicketStride, &sh_ticket);
  if (chunk >= chunks) {  // tickets not reset before the launch: do nothing
    if (threadIdx.x == 0) atomicOr(err, 2u);
    return;
  }
  const int64_t Tn = RAGGED ? (int64_t)g.len[node] : g.T;
  if (RAGGED && chunk >= comp_chunks_of(Tn)) return;  // past the node's length
  const Coef k = load_coef(P, slot);
  const int t0 = chunk * kChunk;
  stage<false, RAGGED>(g, node, t0, sl, sr);
  __syncthreads();
  const int i0 = seg_base(threadIdx.x);  // this thread's kPer samples
  double B = 0.0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) B = fma(k.a, B, k.b * energy(sl, sr, i0 + i));
  double total;
  const double E0 = chunk_scan<false>(B, k, wtot, total);
  uint64_t* tots = agg + (int64_t)ws * chunks;
  if (threadIdx.x == 0) publish(tots + chunk, total);
  const double cin = chunk_carry<false>(tots, chunk, chunks, k, err, g.wait_polls, red);
  if (threadIdx.x == 0) carry[(int64_t)ws * chunks + chunk] = cin;
  double s = fma(pow_a8(k, scan_index(false)), cin, E0);
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    s = fma(k.a, s, k.b * energy(sl, sr, i0 + i));
    const Curve cv = curve<false, GATE>(ln_f((float)(s + kEps)), k);
    const float gam = exp_f(cv.e);
    sl[i0 + i] = gam * sl[i0 + i];
    sr[i0 + i] = gam * sr[i0 + i];
  }
  __syncthreads();
  store_chunk(U + (int64_t)node * 2 * g.T, g.T, Tn, t0, sl, sr);
}

// ---- adjoint ----------------------------------------------------------------------------------

template <bool RAGGED, bool GATE>
__global__ __launch_bounds__(kBlock) void comp_bwd_kernel(GraphView g, float* dU, const float* P,
                                                          int node_begin, int n_nodes, int chunks, int ws_off,
                                                          const double* carry, uint64_t* ragg,
                                                          double* part, unsigned* ticket,
                                                          unsigned* err) {
  __shared__ float ul[kLdsChunk], ur[kLdsChunk], yl[kLdsChunk], yr[kLdsChunk];
  __shared__ double wtot[4], red[4];
  __shared__ int sh_ticket;
  const int node = node_begin + block_node(g, n_nodes, chunks);
  const int slot = g.param_row[node];  // row in P
  const int ws = slot + ws_off;         // row of the dynamics workspace (compressors, then gates)
  const int tk = take_ticket(ticket + (int64_t)ws * kCompTicketStride, &sh_ticket);
  if (tk >= chunks) {  // tickets not reset before the launch: do nothing
    if (threadIdx.x == 0) atomicOr(err, 2u);
    return;
  }
  const int64_t Tn = RAGGED ? (int64_t)g.len[node] : g.T;
  const int chunks_n = RAGGED ? comp_chunks_of(Tn) : chunks;
  if (RAGGED && tk >= chunks_n) {  // past the node's length: this ticket zeroes one unused partial slot
    if (threadIdx.x < 4) part[((int64_t)ws * chunks + tk) * 4 + threadIdx.x] = 0.0;
    return;
  }
  const int chunk = chunks_n - 1 - tk;
  const Coef k = load_coef(P, slot);
  const int t0 = chunk * kChunk;
  stage<false, RAGGED>(g, node, t0, ul, ur);
  stage<true, RAGGED>(g, node, t0, yl, yr);
  __syncthreads();
  const int i0 = seg_base(threadIdx.x);  // this thread's kPer samples
  // envelope rebuilt from the forward carry
  double B = 0.0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) B = fma(k.a, B, k.b * energy(ul, ur, i0 + i));
  double total;
  const double E0 = chunk_scan<false>(B, k, wtot, total);
  const double E = fma(pow_a8(k, scan_index(false)), carry[(int64_t)ws * chunks + chunk], E0);
  // First pass (forward over the thread's samples): envelope, gain and the local adjoint terms.
  // What the reverse pass needs is written back over the thread's own LDS slots: ul <- g[t-1] -
  // x[t], ur <- u_l + u_r, yl/yr <- gain * ybar.
  float gbar[kPer];
  double accT = 0.0, accW = 0.0, accR = 0.0;
  {
    double s = E;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int idx = i0 + i;
      const float u_l = ul[idx], u_r = ur[idx];
      const float m = u_l + u_r;
      const double x = (double)(m * m);  // as in energy()
      const double sprev = s;
      s = fma(k.a, s, k.b * x);
      const float gs = (float)(s + kEps);
      const Curve cv = curve<true, GATE>(ln_f(gs), k);
      const float gam = exp_f(cv.e);
      const float y_l = yl[idx], y_r = yr[idx];
      const float rho = gam * (y_l * u_l + y_r * u_r);
      gbar[i] = rho * cv.dG / gs;
      accT += (double)(rho * cv.dT);
      accW += (double)(rho * cv.dW);
      accR += (double)(rho * cv.dR);
      ul[idx] = (float)(sprev - x);
      ur[idx] = m;
      yl[idx] = gam * y_l;
      yr[idx] = gam * y_r;
    }
  }
  // reverse recursion lambda[t] = gbar[t] + a lambda[t+1]
  double R = 0.0;
#pragma unroll
  for (int i = kPer - 1; i >= 0; --i) R = fma(k.a, R, (double)gbar[i]);
  double rtotal;
  const double L0 = chunk_scan<true>(R, k, wtot, rtotal);
  uint64_t* rtots = ragg + (int64_t)ws * chunks;
  if (threadIdx.x == 0) publish(rtots + chunk, rtotal);
  const double rin = chunk_carry<true>(rtots, chunk, chunks_n, k, err, g.wait_polls, red);  // own chunks
  double lam = fma(pow_a8(k, scan_index(true)), rin, L0);
  double accA = 0.0;
#pragma unroll
  for (int i = kPer - 1; i >= 0; --i) {
    const int idx = i0 + i;
    lam = fma(k.a, lam, (double)gbar[i]);
    accA += lam * (double)ul[idx];
    const float mid = (float)(2.0 * k.b * lam) * ur[idx];
    yl[idx] += mid;
    yr[idx] += mid;
  }
  const double sA = block_sum<double>(accA, red);
  const double sT = block_sum<double>(accT, red);
  const double sW = block_sum<double>(accW, red);
  const double sR = block_sum<double>(accR, red);
  if (threadIdx.x == 0) {
    double* p = part + ((int64_t)ws * chunks + chunk) * 4;
    p[0] = sA;
    p[1] = sT;
    p[2] = sW;
    p[3] = sR;
  }
  store_chunk(dU + (int64_t)node * 2 * g.T, g.T, Tn, t0, yl, yr);
}

// Reset the published totals to "not ready" and the per-node tickets to 0 before a pass.
__global__ __launch_bounds__(kBlock) void comp_reset_kernel(uint64_t* tot, int64_t n,
                                                            unsigned* tickets, int n_tickets) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) tot[i] = kNotReady;
  if (i < n_tickets) tickets[i] = 0u;
}

}  // namespace

int comp_chunks(int64_t T) { return (int)((T + kChunk - 1) / kChunk); }

hipError_t launch_comp_reset(uint64_t* tot, int64_t n, unsigned* tickets, int n_tickets,
                             hipStream_t s) {
  const int64_t m = n > n_tickets ? n : n_tickets;
  if (m <= 0) return hipSuccess;
  comp_reset_kernel<<<(unsigned)((m + kBlock - 1) / kBlock), kBlock, 0, s>>>(tot, n, tickets,
                                                                              n_tickets);
  return hipGetLastError();
}

template <bool RAGGED, bool GATE>
static void launch_fwd_t(const GraphView& g, float* U, const float* P, int node_begin,
                         int n_nodes, int chunks, int ws_off, uint64_t* agg, double* carry,
                         unsigned* ticket, unsigned* err, hipStream_t s) {
  comp_fwd_kernel<RAGGED, GATE><<<(unsigned)(chunks * n_nodes), kBlock, 0, s>>>(
      g, U, P, node_begin, n_nodes, chunks, ws_off, agg, carry, ticket, err);
}

template <bool RAGGED, bool GATE>
static void launch_bwd_t(const GraphView& g, float* dU, const float* P, int node_begin,
                         int n_nodes, int chunks, int ws_off, const double* carry, uint64_t* ragg,
                         double* part, unsigned* ticket, unsigned* err, hipStream_t s) {
  comp_bwd_kernel<RAGGED, GATE><<<(unsigned)(chunks * n_nodes), kBlock, 0, s>>>(
      g, dU, P, node_begin, n_nodes, chunks, ws_off, carry, ragg, part, ticket, err);
}

// Per-node lengths and the noisegate curve get their own instantiations, so the uniform
// compressor carries no code for either.
hipError_t launch_comp_fwd(const GraphView& g, float* U, const float* P, int node_begin,
                           int n_nodes, int ws_off, bool gate, uint64_t* agg, double* carry,
                           unsigned* ticket, unsigned* err, hipStream_t s) {
  const int chunks = comp_chunks(g.T);
  if (g.len)
    (gate ? launch_fwd_t<true, true> : launch_fwd_t<true, false>)(
        g, U, P, node_begin, n_nodes, chunks, ws_off, agg, carry, ticket, err, s);
  else
    (gate ? launch_fwd_t<false, true> : launch_fwd_t<false, false>)(
        g, U, P, node_begin, n_nodes, chunks, ws_off, agg, carry, ticket, err, s);
  return hipGetLastError();
}

hipError_t launch_comp_bwd(const GraphView& g, float* dU, const float* P, int node_begin,
                           int n_nodes, int ws_off, bool gate, const double* carry,
                           uint64_t* ragg, double* part, unsigned* ticket, unsigned* err,
                           hipStream_t s) {
  const int chunks = comp_chunks(g.T);
  if (g.len)
    (gate ? launch_bwd_t<true, true> : launch_bwd_t<true, false>)(
        g, dU, P, node_begin, n_nodes, chunks, ws_off, carry, ragg, part, ticket, err, s);
  else
    (gate ? launch_bwd_t<false, true> : launch_bwd_t<false, false>)(
        g, dU, P, node_begin, n_nodes, chunks, ws_off, carry, ragg, part, ticket, err, s);
  return hipGetLastError();
}

}  // namespace grafx
