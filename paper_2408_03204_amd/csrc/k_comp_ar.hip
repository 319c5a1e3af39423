// Compressor with distinct attack and release ballistics (paper Sec. 3 "Compressor": Eq. 8 with
// alpha[t] = alpha_a while the envelope rises and alpha_r otherwise, then the knee and gain of
// Eqs. 10-12), parallel across nodes and time chunks.
//
// The branch x[t] > g[t-1] makes the recursion non-linear, but for a fixed branch pattern it is a
// linear recursion with a per-sample coefficient, g[t] = a_t g[t-1] + (1 - a_t) x[t], which a
// chunked scan of affine maps (A, B): g -> A g + B computes exactly. The forward kernel iterates
// on the pattern: pass 0 takes every sample as release; each pass scans with its pattern and
// derives the next one from the envelope it produced. If a pass leaves the pattern of a time
// prefix unchanged, that prefix is exact: at the first sample where a pattern is wrong, the
// envelope before it is exact, so the next pattern corrects that sample and differs there.
// Hence a chunk is final once its own pattern and those of all earlier chunks were left unchanged
// by the previous pass (random signals settle in 3-8 passes). Each pass publishes, per chunk, its
// map and whether the chunk's pattern changed in the previous pass, so one round of publication
// serves both the entering state and the settling test. Chunk c of pass k waits only for words of
// earlier chunks of pass k: a chunk that settles fills its later pass slots with its final map, so
// no wait depends on a later chunk and every wait ends. A chunk still unsettled
// after the last pass takes the exact state entering it from the final maps of the earlier
// chunks and runs the literal recursion over its 3072 samples on one thread, which settles it.
//
// Chunk geometry, tickets, publication and staging are those of the compressor with one
// ballistics constant (256 threads x 12 consecutive samples, one 64-bit relaxed device-scope
// atomic per published value over a "not ready" sentinel, bounded waits that poison their result
// and set an error bit). A thread's map is the composition of its 12 sample maps; a Kogge-Stone
// scan across the wave and a fold across the 4 waves give every thread the map from the chunk
// start to its first sample. The state entering a chunk composes the published maps of the
// earlier chunks in time order: contiguous ranges per thread, then the same block scan, so the
// arithmetic depends only on the node's data (deterministic, independent of the schedule).
//
// Adjoint (rho = sum_c ybar_c y_c, e = G_y - G_u, the pattern fixed as in the forward call):
//   gbar = rho de/dG_u / (g + 1e-8);  lambda[t] = gbar[t] + mu[t+1],  mu[t] = a_t lambda[t]
//   (a reverse scan of the maps mu[t+1] -> a_t mu[t+1] + a_t gbar[t]);
//   ubar_c = gamma ybar_c + 2 (u_l + u_r)(1 - a_t) lambda;
//   dL/d alpha_a (alpha_r) = sum of lambda[t] (g[t-1] - x[t]) over the attack (release) samples;
//   dL/d(T, W, R) = sum rho de/d(T, W, R).
// The forward call keeps each chunk's entering state and its final pattern (12 bits per thread).
#include "device_common.h"
#include "dynamics.h"
#include "grafx_internal.h"
#include "kernels.h"

namespace grafx {
namespace {

using namespace dyn;

struct CoefAR {
  double aa, ar, ba, br;  // alpha_a, alpha_r, 1 - alpha_a, 1 - alpha_r
  float thr, knee;        // T, W
  float c, g1;            // 1/R - 1, 1 - R
  float inv2w, inv4w;     // 1/(2W), 1/(4W)
  float invR2;            // 1/R^2
};

__device__ __forceinline__ CoefAR load_coef_ar(const float* P, int slot) {
  CoefAR k;
  const float* p = P + (int64_t)slot * kArParams;
  k.aa = (double)p[0];
  k.ar = (double)p[1];
  k.ba = 1.0 - k.aa;
  k.br = 1.0 - k.ar;
  k.thr = p[2];
  k.knee = p[3];
  const float R = p[4];
  k.c = 1.0f / R - 1.0f;
  k.g1 = 1.0f - R;
  k.inv2w = k.knee > 0.f ? 1.0f / (2.f * k.knee) : 0.f;
  k.inv4w = k.knee > 0.f ? 1.0f / (4.f * k.knee) : 0.f;
  k.invR2 = 1.0f / (R * R);
  return k;
}

// Affine map s -> A s + B.
struct Aff {
  double A, B;
};

// g after f (f applied first).
__device__ __forceinline__ Aff after(const Aff& g, const Aff& f) {
  return {g.A * f.A, fma(g.A, f.B, g.B)};
}

// Map of a thread's kPer samples under its branch pattern (bit i set: sample i is attack).
__device__ __forceinline__ Aff thread_map(const float* x, int pat, const CoefAR& k) {
  Aff f = {1.0, 0.0};
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const bool up = (pat >> i) & 1;
    const double a = up ? k.aa : k.ar;
    f.A *= a;
    f.B = fma(a, f.B, (up ? k.ba : k.br) * (double)x[i]);
  }
  return f;
}

// Scan of the threads' maps in time order (REV: thread kBlock-1 first). Returns the composition
// of the maps of the threads before this one (identity for the first); `total` receives the
// composition over the whole block (every thread).
template <bool REV>
__device__ __forceinline__ Aff aff_scan(Aff f, Aff* wtot, Aff& total) {
  const int lane0 = threadIdx.x & 63, w0 = threadIdx.x >> 6;
  const int lane = REV ? 63 - lane0 : lane0;
  const int w = REV ? 3 - w0 : w0;
  Aff S = f;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    Aff o;
    o.A = REV ? __shfl_down(S.A, 1 << d, 64) : __shfl_up(S.A, 1 << d, 64);
    o.B = REV ? __shfl_down(S.B, 1 << d, 64) : __shfl_up(S.B, 1 << d, 64);
    if (lane >= (1 << d)) S = after(S, o);
  }
  Aff ex;
  ex.A = REV ? __shfl_down(S.A, 1, 64) : __shfl_up(S.A, 1, 64);
  ex.B = REV ? __shfl_down(S.B, 1, 64) : __shfl_up(S.B, 1, 64);
  if (lane == 0) ex = {1.0, 0.0};
  __syncthreads();
  if (lane == 63) wtot[w] = S;
  __syncthreads();
  Aff pre = {1.0, 0.0}, all = {1.0, 0.0};
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (v < w) pre = after(wtot[v], pre);
    all = after(wtot[v], all);
  }
  total = all;
  return after(ex, pre);
}

// Composition, in order, of n published maps: map r (r = 0 first) sits at words
// base + idx(r) * stride (A) and + 1 (B), idx(r) = r (FWD) or n - 1 - r. Thread t composes a
// contiguous range of r, the block scan composes the ranges. Returns B of the composition, i.e.
// the state it gives from a zero start.
template <bool FWD>
__device__ __forceinline__ double fold_maps(uint64_t* base, int stride, int n, unsigned* err,
                                            int polls, Aff* wtot) {
  const int per = (n + kBlock - 1) / kBlock;
  const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
  Aff m = {1.0, 0.0};
  for (int r = lo; r < hi; ++r) {
    uint64_t* w = base + (int64_t)(FWD ? r : n - 1 - r) * stride;
    const Aff o = {await_total(w, err, polls), await_total(w + 1, err, polls)};
    m = after(o, m);
  }
  Aff total;
  aff_scan<false>(m, wtot, total);
  return total.B;
}

// fold_maps<true> over the pass rows (A, B, flag) of the chunks before `chunk`, which also
// returns in `all` whether `own` and every earlier chunk's flag are set (block-uniform).
__device__ __forceinline__ double fold_maps_flags(uint64_t* row, int chunk, unsigned* err,
                                                  int polls, Aff* wtot, bool own, bool& all) {
  const int per = (chunk + kBlock - 1) / kBlock;
  const int lo = min(chunk, (int)threadIdx.x * per), hi = min(chunk, lo + per);
  Aff m = {1.0, 0.0};
  bool ok = own;
  for (int r = lo; r < hi; ++r) {
    uint64_t* w = row + (int64_t)r * 3;
    const Aff o = {await_total(w, err, polls), await_total(w + 1, err, polls)};
    ok = ok && await_total(w + 2, err, polls) == 1.0;
    m = after(o, m);
  }
  all = __syncthreads_and(ok) != 0;
  Aff total;
  aff_scan<false>(m, wtot, total);
  return total.B;
}

// ---- forward ----------------------------------------------------------------------------------

// pslot: [n_ar][kArPasses][chunks][3] (A, B, stable flag) per pass; fin: [n_ar][chunks][2] final
// maps; carry: [n_ar][chunks] entering states; pats: [n_ar][chunks][kBlock] final patterns.
template <bool RAGGED>
__global__ __launch_bounds__(kBlock) void comp_ar_fwd_kernel(
    GraphView g, float* U, const float* P, int node_begin, int n_nodes, int chunks, int max_pass,
    uint64_t* pslot, uint64_t* fin, double* carry, uint16_t* pats, unsigned* ticket,
    unsigned* err) {
  __shared__ float sl[kLdsChunk], sr[kLdsChunk];
  __shared__ Aff wtot[4];
  __shared__ uint16_t sh_pat[kBlock];
  __shared__ int sh_ticket;
  const int node = node_begin + block_node(g, n_nodes, chunks);
  const int slot = g.param_row[node];
  const int chunk = take_ticket(ticket + (int64_t)slot * kCompTicketStride, &sh_ticket);
  if (chunk >= chunks) {  // tickets not reset before the launch: do nothing
    if (threadIdx.x == 0) atomicOr(err, 2u);
    return;
  }
  const int64_t Tn = RAGGED ? (int64_t)g.len[node] : g.T;
  if (RAGGED && chunk >= comp_chunks_of(Tn)) return;  // past the node's length
  const CoefAR k = load_coef_ar(P, slot);
  const int t0 = chunk * kChunk;
  stage<false, RAGGED>(g, node, t0, sl, sr);
  __syncthreads();
  const int i0 = seg_base(threadIdx.x);  // this thread's kPer samples
  float x[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const float m = sl[i0 + i] + sr[i0 + i];
    x[i] = m * m;
  }
  uint64_t* ps = pslot + (int64_t)slot * kArPasses * chunks * 3;
  uint64_t* fn = fin + (int64_t)slot * chunks * 2;
  int pat = 0;   // pass 0: every sample taken as release
  int prev = 0;  // the pattern of the previous pass
  bool done = false;
  double cin = 0.0;
  Aff tot = {1.0, 0.0};
  for (int pass = 0; pass < max_pass && !done; ++pass) {
    const Aff ex = aff_scan<false>(thread_map(x, pat, k), wtot, tot);
    // did the previous pass leave this chunk's pattern unchanged?
    const bool same = __syncthreads_and(pass > 0 && pat == prev) != 0;
    uint64_t* row = ps + (int64_t)pass * chunks * 3;
    if (threadIdx.x == 0) {
      publish(row + (int64_t)chunk * 3, tot.A);
      publish(row + (int64_t)chunk * 3 + 1, tot.B);
      publish(row + (int64_t)chunk * 3 + 2, same ? 1.0 : 0.0);
    }
    bool all_same;
    cin = fold_maps_flags(row, chunk, err, g.wait_polls, wtot, same, all_same);
    if (all_same) {  // the pattern of this pass is exact up to the chunk's end, and so is cin
      done = true;
      for (int q = pass + 1 + (int)threadIdx.x; q < max_pass; q += kBlock) {
        uint64_t* r = ps + ((int64_t)q * chunks + chunk) * 3;
        publish(r, tot.A);
        publish(r + 1, tot.B);
        publish(r + 2, 1.0);
      }
    } else {  // the next pattern, from the envelope of this pass
      double s = fma(ex.A, cin, ex.B);
      int np = 0;
#pragma unroll
      for (int i = 0; i < kPer; ++i) {
        const double xi = (double)x[i];
        np |= (int)(xi > s) << i;
        const bool up = (pat >> i) & 1;
        s = fma(up ? k.aa : k.ar, s, (up ? k.ba : k.br) * xi);
      }
      prev = pat;
      pat = np;
    }
  }
  if (!done) {  // serial fallback from the exact entering state
    cin = fold_maps<true>(fn, 2, chunk, err, g.wait_polls, wtot);
    if (threadIdx.x == 0) {
      double s = cin;
      for (int j = 0; j < kBlock; ++j) {
        int p = 0;
        for (int i = 0; i < kPer; ++i) {
          const float m = sl[seg_base(j) + i] + sr[seg_base(j) + i];
          const double xi = (double)(m * m);
          const bool up = xi > s;
          p |= (int)up << i;
          s = fma(up ? k.aa : k.ar, s, (up ? k.ba : k.br) * xi);
        }
        sh_pat[j] = (uint16_t)p;
      }
    }
    __syncthreads();
    pat = sh_pat[threadIdx.x];
  }
  const Aff ex = aff_scan<false>(thread_map(x, pat, k), wtot, tot);
  if (threadIdx.x == 0) {
    publish(fn + (int64_t)chunk * 2, tot.A);
    publish(fn + (int64_t)chunk * 2 + 1, tot.B);
    carry[(int64_t)slot * chunks + chunk] = cin;
  }
  pats[((int64_t)slot * chunks + chunk) * kBlock + threadIdx.x] = (uint16_t)pat;
  double s = fma(ex.A, cin, ex.B);
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const bool up = (pat >> i) & 1;
    s = fma(up ? k.aa : k.ar, s, (up ? k.ba : k.br) * (double)x[i]);
    const Curve cv = comp_curve<false>(ln_f((float)(s + kEps)), k);
    const float gam = exp_f(cv.e);
    sl[i0 + i] = gam * sl[i0 + i];
    sr[i0 + i] = gam * sr[i0 + i];
  }
  __syncthreads();
  store_chunk(U + (int64_t)node * 2 * g.T, g.T, Tn, t0, sl, sr);
}

// ---- adjoint ----------------------------------------------------------------------------------

// ragg: [n_ar][chunks][2] published reverse maps; part: [n_ar][chunks][5] parameter partials.
// Capped at 168 VGPRs (three waves per SIMD instead of two, with a few values spilled): measured
// 6 % faster on the attack/release console than uncapped; the forward kernel, capped likewise at
// four waves, spilled in its pass loop and was slower.
template <bool RAGGED>
__global__ __launch_bounds__(kBlock, 3) void comp_ar_bwd_kernel(
    GraphView g, float* dU, const float* P, int node_begin, int n_nodes, int chunks,
    const double* carry, const uint16_t* pats, uint64_t* ragg, double* part, unsigned* ticket,
    unsigned* err) {
  __shared__ float ul[kLdsChunk], ur[kLdsChunk], yl[kLdsChunk], yr[kLdsChunk];
  __shared__ Aff wtot[4];
  __shared__ double red[4];
  __shared__ int sh_ticket;
  const int node = node_begin + block_node(g, n_nodes, chunks);
  const int slot = g.param_row[node];
  const int tk = take_ticket(ticket + (int64_t)slot * kCompTicketStride, &sh_ticket);
  if (tk >= chunks) {  // tickets not reset before the launch: do nothing
    if (threadIdx.x == 0) atomicOr(err, 2u);
    return;
  }
  const int64_t Tn = RAGGED ? (int64_t)g.len[node] : g.T;
  const int chunks_n = RAGGED ? comp_chunks_of(Tn) : chunks;
  if (RAGGED && tk >= chunks_n) {  // past the node's length: zero one unused partial slot
    if (threadIdx.x < kArParams) part[((int64_t)slot * chunks + tk) * kArParams + threadIdx.x] = 0.0;
    return;
  }
  const int chunk = chunks_n - 1 - tk;
  const CoefAR k = load_coef_ar(P, slot);
  const int t0 = chunk * kChunk;
  stage<false, RAGGED>(g, node, t0, ul, ur);
  stage<true, RAGGED>(g, node, t0, yl, yr);
  __syncthreads();
  const int i0 = seg_base(threadIdx.x);  // this thread's kPer samples
  const int pat = pats[((int64_t)slot * chunks + chunk) * kBlock + threadIdx.x];
  float x[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const float m = ul[i0 + i] + ur[i0 + i];
    x[i] = m * m;
  }
  Aff tot;
  const Aff ex = aff_scan<false>(thread_map(x, pat, k), wtot, tot);
  // First pass (forward over the thread's samples): envelope, gain and the local adjoint terms;
  // ul <- g[t-1] - x[t], ur <- u_l + u_r, yl/yr <- gain * ybar over the thread's own LDS slots.
  float gbar[kPer];
  double accT = 0.0, accW = 0.0, accR = 0.0;
  {
    double s = fma(ex.A, carry[(int64_t)slot * chunks + chunk], ex.B);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int idx = i0 + i;
      const float u_l = ul[idx], u_r = ur[idx];
      const double xi = (double)x[i];
      const double sprev = s;
      const bool up = (pat >> i) & 1;
      s = fma(up ? k.aa : k.ar, s, (up ? k.ba : k.br) * xi);
      const float gs = (float)(s + kEps);
      const Curve cv = comp_curve<true>(ln_f(gs), k);
      const float gam = exp_f(cv.e);
      const float y_l = yl[idx], y_r = yr[idx];
      const float rho = gam * (y_l * u_l + y_r * u_r);
      gbar[i] = rho * cv.dG / gs;
      accT += (double)(rho * cv.dT);
      accW += (double)(rho * cv.dW);
      accR += (double)(rho * cv.dR);
      ul[idx] = (float)(sprev - xi);
      ur[idx] = u_l + u_r;
      yl[idx] = gam * y_l;
      yr[idx] = gam * y_r;
    }
  }
  // reverse maps mu[t+1] -> a_t mu[t+1] + a_t gbar[t] over the thread's samples, last first
  Aff m = {1.0, 0.0};
#pragma unroll
  for (int i = kPer - 1; i >= 0; --i) {
    const double a = ((pat >> i) & 1) ? k.aa : k.ar;
    m = after(Aff{a, a * (double)gbar[i]}, m);
  }
  Aff rtot;
  const Aff rex = aff_scan<true>(m, wtot, rtot);
  uint64_t* rn = ragg + (int64_t)slot * chunks * 2;
  if (threadIdx.x == 0) {
    publish(rn + (int64_t)chunk * 2, rtot.A);
    publish(rn + (int64_t)chunk * 2 + 1, rtot.B);
  }
  // maps of the later chunks of this node, the last one first
  const double rin = fold_maps<false>(rn + (int64_t)(chunk + 1) * 2, 2, chunks_n - 1 - chunk, err,
                                      g.wait_polls, wtot);
  double mu = fma(rex.A, rin, rex.B);
  double accAa = 0.0, accAr = 0.0;
#pragma unroll
  for (int i = kPer - 1; i >= 0; --i) {
    const int idx = i0 + i;
    const bool up = (pat >> i) & 1;
    const double lam = (double)gbar[i] + mu;
    const double d = lam * (double)ul[idx];
    if (up)
      accAa += d;
    else
      accAr += d;
    const float mid = (float)(2.0 * (up ? k.ba : k.br) * lam) * ur[idx];
    yl[idx] += mid;
    yr[idx] += mid;
    mu = (up ? k.aa : k.ar) * lam;
  }
  const double sAa = block_sum<double>(accAa, red);
  const double sAr = block_sum<double>(accAr, red);
  const double sT = block_sum<double>(accT, red);
  const double sW = block_sum<double>(accW, red);
  const double sR = block_sum<double>(accR, red);
  if (threadIdx.x == 0) {
    double* p = part + ((int64_t)slot * chunks + chunk) * kArParams;
    p[0] = sAa;
    p[1] = sAr;
    p[2] = sT;
    p[3] = sW;
    p[4] = sR;
  }
  store_chunk(dU + (int64_t)node * 2 * g.T, g.T, Tn, t0, yl, yr);
}

}  // namespace

hipError_t launch_comp_ar_fwd(const GraphView& g, float* U, const float* P, int node_begin,
                              int n_nodes, int max_pass, uint64_t* pslot, uint64_t* fin,
                              double* carry, uint16_t* pats, unsigned* ticket, unsigned* err,
                              hipStream_t s) {
  if (max_pass < 1 || max_pass > kArPasses) return hipErrorInvalidValue;
  const int chunks = comp_chunks(g.T);
  const unsigned grid = (unsigned)(chunks * n_nodes);
  if (g.len)
    comp_ar_fwd_kernel<true><<<grid, kBlock, 0, s>>>(g, U, P, node_begin, n_nodes, chunks,
                                                     max_pass, pslot, fin, carry, pats, ticket,
                                                     err);
  else
    comp_ar_fwd_kernel<false><<<grid, kBlock, 0, s>>>(g, U, P, node_begin, n_nodes, chunks,
                                                      max_pass, pslot, fin, carry, pats, ticket,
                                                      err);
  return hipGetLastError();
}

hipError_t launch_comp_ar_bwd(const GraphView& g, float* dU, const float* P, int node_begin,
                              int n_nodes, const double* carry, const uint16_t* pats,
                              uint64_t* ragg, double* part, unsigned* ticket, unsigned* err,
                              hipStream_t s) {
  const int chunks = comp_chunks(g.T);
  const unsigned grid = (unsigned)(chunks * n_nodes);
  if (g.len)
    comp_ar_bwd_kernel<true><<<grid, kBlock, 0, s>>>(g, dU, P, node_begin, n_nodes, chunks, carry,
                                                     pats, ragg, part, ticket, err);
  else
    comp_ar_bwd_kernel<false><<<grid, kBlock, 0, s>>>(g, dU, P, node_begin, n_nodes, chunks, carry,
                                                      pats, ragg, part, ticket, err);
  return hipGetLastError();
}

}  // namespace grafx
