// Fused gather-sum -> pointwise processor -> store, for one schedule step (paper Algorithm 1:
// Gather, Aggregate, Process, Store of one iteration), and the matching adjoint step.
//
// Types: mix / out (identity, Eq. 1b only), gain_pan (Eq. 2), imager (Eq. 3), tanh distortion.
// One block of 256 threads covers 1024 x UN samples of one node (both channels), UN = 1, 2 or 4
// being a tuning setting of the schedule; blockIdx.y picks the node inside the step. Thread j
// covers samples 4j..4j+3 of each 1024-sample part of the tile: with T and every node
// length multiples of 4, rows are 16-byte aligned and it moves one float4 per channel and input;
// otherwise it moves the 4 samples one by one. Inputs are read through raw buffer resources sized to their node's
// length, so samples past an input's length read as zero without a branch, and are summed in
// original edge order, so a node's arithmetic does not depend on the step it was batched into.
// A node's own samples past its length are neither computed nor stored.
#include "device_common.h"
#include "grafx_internal.h"
#include "kernels.h"

namespace grafx {
namespace {

constexpr int kTile = 1024;

struct Gains {
  float e0, e1;
};

template <int TYPE>
__device__ __forceinline__ Gains load_gains(const float* P, int row) {
  Gains g{1.f, 1.f};
  if constexpr (TYPE == GRAFX_GAIN_PAN) {
    g.e0 = expf(P[2 * row]);
    g.e1 = expf(P[2 * row + 1]);
  } else if constexpr (TYPE == GRAFX_IMAGER || TYPE == GRAFX_TANH) {
    g.e0 = expf(P[row]);
  }
  return g;
}

template <int TYPE>
__device__ __forceinline__ void fwd_op(float& l, float& r, Gains k) {
  if constexpr (TYPE == GRAFX_GAIN_PAN) {
    l *= k.e0;
    r *= k.e1;
  } else if constexpr (TYPE == GRAFX_IMAGER) {
    const float m = l + r, s = k.e0 * (l - r);
    l = 0.5f * (m + s);
    r = 0.5f * (m - s);
  } else if constexpr (TYPE == GRAFX_TANH) {
    l = tanhf(k.e0 * l);
    r = tanhf(k.e0 * r);
  }
}

// Streaming store of 4 floats (16-byte aligned): marked non-temporal, since a step's output rows
// are read back only by later steps, long after the caches have turned over.
typedef float v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void nt_store4(float* p, float a, float b, float c, float d) {
  __builtin_nontemporal_store(v4f{a, b, c, d}, reinterpret_cast<v4f*>(p));
}

// Input rows are read once per consumer: loads marked non-temporal (cache policy bit 1).
__device__ __forceinline__ float4 bload4(__amdgpu_buffer_rsrc_t r, int idx) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, idx * 4, 0, 2));
}

// n (4 or 1) consecutive floats of a row through a length-bounded buffer resource
template <bool V4>
__device__ __forceinline__ void bload_n(__amdgpu_buffer_rsrc_t r, int idx, float* out) {
  if constexpr (V4) {
    const float4 a = bload4(r, idx);
    out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
  } else {
    out[0] = bload(r, idx);
  }
}

template <int TYPE, bool V4, int UN>
__global__ __launch_bounds__(kBlock) void pointwise_fwd_kernel(GraphView g, float* U,
                                                               const float* P, int node_begin) {
  const int node = node_begin + blockIdx.y;
  const int64_t T = g.T, Tn = node_len(g, node);
  const int64_t base = (int64_t)blockIdx.x * (kTile * UN);
  if (base >= Tn) return;  // tile past the node's length (uniform over the block)
  const Gains k = load_gains<TYPE>(P, g.param_row[node]);
  const int e0 = g.in_ptr[node], e1 = g.in_ptr[node + 1];
  float* y = U + (int64_t)node * 2 * T;
  // thread j covers samples base + kTile u + 4 j .. + 3 for u < UN; every load of an input row
  // is issued before any is summed (samples past an input's length read as zero)
  float l[UN][4], r[UN][4];
#pragma unroll
  for (int u = 0; u < UN; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) l[u][q] = r[u][q] = 0.f;
  for (int e = e0; e < e1; ++e) {
    const int src = g.in_src[e];
    const float* row = out_row(g, src);
    const int64_t Ls = node_len(g, src);
    const auto rl = row_rsrc(row, Ls), rr = row_rsrc(row + T, Ls);
    float a[UN][4], b[UN][4];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int t = (int)(base + kTile * u + 4 * threadIdx.x);
      if constexpr (V4) {
        const float4 x = bload4(rl, t), z = bload4(rr, t);
        a[u][0] = x.x; a[u][1] = x.y; a[u][2] = x.z; a[u][3] = x.w;
        b[u][0] = z.x; b[u][1] = z.y; b[u][2] = z.z; b[u][3] = z.w;
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          a[u][q] = bload(rl, t + q);
          b[u][q] = bload(rr, t + q);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < UN; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        l[u][q] += a[u][q];
        r[u][q] += b[u][q];
      }
  }
#pragma unroll
  for (int u = 0; u < UN; ++u) {
    const int64_t t = base + kTile * u + 4 * threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) fwd_op<TYPE>(l[u][q], r[u][q], k);
    if constexpr (V4) {
      if (t < Tn) {
        nt_store4(y + t, l[u][0], l[u][1], l[u][2], l[u][3]);
        nt_store4(y + T + t, r[u][0], r[u][1], r[u][2], r[u][3]);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (t + q < Tn) {
          y[t + q] = l[u][q];
          y[T + t + q] = r[u][q];
        }
    }
  }
}

// Adjoint of one pointwise step. `dst` receives the input adjoint (dU, or dS for the input step,
// whose rows are indexed the same way). Parameter-gradient partials (one per block and
// parameter, double) go to part[(slot * tiles + tile) * NP + j].
template <bool V4>
__device__ __forceinline__ void load_n(const float* p, float* out) {
  if constexpr (V4) {
    const v4f a = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
    out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
  } else {
    out[0] = *p;
  }
}

template <bool V4>
__device__ __forceinline__ void store_n(float* p, const float* v) {
  if constexpr (V4) nt_store4(p, v[0], v[1], v[2], v[3]);
  else *p = v[0];
}

template <int TYPE>
struct AdjOp {
  static constexpr int NP = TYPE == GRAFX_GAIN_PAN ? 2 : (TYPE == GRAFX_IMAGER || TYPE == GRAFX_TANH ? 1 : 0);
};

template <int TYPE>
__device__ __forceinline__ void adj_op(float yl, float yr, float ul_in, float ur_in, float& gl,
                                       float& gr, Gains k, float* acc) {
  // yl, yr: node output (gain_pan, imager); ul_in, ur_in: node input (tanh); gl, gr: output
  // adjoint in, input adjoint out
  if constexpr (TYPE == GRAFX_GAIN_PAN) {
    acc[0] += gl * yl;
    acc[1] += gr * yr;
    gl *= k.e0;
    gr *= k.e1;
  } else if constexpr (TYPE == GRAFX_IMAGER) {
    const float mb = 0.5f * (gl + gr), sb = 0.5f * (gl - gr);
    acc[0] += sb * (yl - yr);
    gl = mb + k.e0 * sb;
    gr = mb - k.e0 * sb;
  } else if constexpr (TYPE == GRAFX_TANH) {
    const float al = tanhf(k.e0 * ul_in), ar = tanhf(k.e0 * ur_in);
    gl = gl * k.e0 * (1.f - al * al);
    gr = gr * k.e0 * (1.f - ar * ar);
    acc[0] += gl * ul_in + gr * ur_in;
  }
}

template <int TYPE, bool V4, int UN>
__global__ __launch_bounds__(kBlock) void pointwise_bwd_kernel(GraphView g, float* dst,
                                                               const float* P, int node_begin,
                                                               double* part, int tiles) {
  constexpr int NP = AdjOp<TYPE>::NP;
  const int node = node_begin + blockIdx.y;
  const int64_t T = g.T, Tn = node_len(g, node);
  const int slot = g.param_row[node];
  const Gains k = load_gains<TYPE>(P, slot);
  const int o0 = g.out_ptr[node], o1 = g.out_ptr[node + 1];
  const int i0 = g.in_ptr[node], i1 = g.in_ptr[node + 1];
  const float* yrow = g.U + (int64_t)node * 2 * T;  // used by gain_pan / imager only
  float* d = dst + (int64_t)node * 2 * T;
  float acc[NP > 0 ? NP : 1] = {0.f};
  const int64_t base = (int64_t)blockIdx.x * (kTile * UN);
  constexpr int NV = V4 ? 4 : 1;
  // Thread j covers samples base + kTile u + 4j .. + 3 (u < UN) in both paths, in the same order,
  // so the gradient partials are accumulated identically whichever path a launch takes. Blocks
  // past the node's length still write their (zero) partials.
#pragma unroll
  for (int u = 0; u < UN; ++u) {
    const int64_t t_first = base + kTile * u + 4 * threadIdx.x;
#pragma unroll
    for (int q = 0; q < (V4 ? 1 : 4); ++q) {
      const int64_t t = t_first + q;
      if (t >= Tn) break;
      float gl[NV], gr[NV], yl[NV], yr[NV], ul[NV], ur[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) gl[v] = gr[v] = yl[v] = yr[v] = ul[v] = ur[v] = 0.f;
      for (int e = o0; e < o1; ++e) {
        const int dnode = g.out_dst[e];
        const float* row = adj_row(g, dnode);
        const int64_t Ld = node_len(g, dnode);
        float a[NV], b[NV];
        bload_n<V4>(row_rsrc(row, Ld), (int)t, a);
        bload_n<V4>(row_rsrc(row + T, Ld), (int)t, b);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          gl[v] += a[v];
          gr[v] += b[v];
        }
      }
      if constexpr (TYPE == GRAFX_GAIN_PAN || TYPE == GRAFX_IMAGER) {
        load_n<V4>(yrow + t, yl);
        load_n<V4>(yrow + T + t, yr);
      }
      if constexpr (TYPE == GRAFX_TANH) {
        for (int e = i0; e < i1; ++e) {
          const int src = g.in_src[e];
          const float* row = out_row(g, src);
          const int64_t Ls = node_len(g, src);
          float a[NV], b[NV];
          bload_n<V4>(row_rsrc(row, Ls), (int)t, a);
          bload_n<V4>(row_rsrc(row + T, Ls), (int)t, b);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            ul[v] += a[v];
            ur[v] += b[v];
          }
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) adj_op<TYPE>(yl[v], yr[v], ul[v], ur[v], gl[v], gr[v], k, acc);
      store_n<V4>(d + t, gl);
      store_n<V4>(d + T + t, gr);
    }
  }
  (void)i0;
  (void)i1;
  if constexpr (NP > 0) {
    __shared__ double red[4];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const double s = block_sum<double>((double)acc[j], red);
      if (threadIdx.x == 0) part[((int64_t)slot * tiles + blockIdx.x) * NP + j] = s;
    }
  }
}

// dP[slot][j] = sum over tiles of part[slot][tile][j], fixed order; one launch for every job of
// the list, block b serving slot b of the concatenated slot ranges.
__global__ __launch_bounds__(kBlock) void reduce_partials_kernel(ReduceJobs J) {
  __shared__ double red[4];
  int slot = blockIdx.x, q = 0;
  while (q + 1 < J.n && slot >= J.slots[q]) slot -= J.slots[q++];  // uniform over the block
  const double* part = J.part[q];
  const int tiles = J.tiles[q], np = J.np[q];
  for (int j = 0; j < np; ++j) {
    double s = 0.0;
    for (int i = threadIdx.x; i < tiles; i += kBlock) s += part[((int64_t)slot * tiles + i) * np + j];
    s = block_sum<double>(s, red);
    if (threadIdx.x == 0) J.dP[q][(int64_t)slot * np + j] = (float)s;
  }
}

template <int TYPE, int UN>
void fwd_un(const GraphView& g, float* U, const float* P, int node_begin, int n_nodes,
            hipStream_t s) {
  dim3 grid((unsigned)((g.T + kTile * UN - 1) / (kTile * UN)), (unsigned)n_nodes);
  if (g.vec4)
    pointwise_fwd_kernel<TYPE, true, UN><<<grid, kBlock, 0, s>>>(g, U, P, node_begin);
  else
    pointwise_fwd_kernel<TYPE, false, UN><<<grid, kBlock, 0, s>>>(g, U, P, node_begin);
}

template <int TYPE>
hipError_t launch_fwd_t(const GraphView& g, float* U, const float* P, int node_begin,
                        int n_nodes, hipStream_t s) {
  switch (g.pw_unroll) {
    case 2: fwd_un<TYPE, 2>(g, U, P, node_begin, n_nodes, s); break;
    case 4: fwd_un<TYPE, 4>(g, U, P, node_begin, n_nodes, s); break;
    default: fwd_un<TYPE, 1>(g, U, P, node_begin, n_nodes, s); break;
  }
  return hipGetLastError();
}

template <int TYPE, int UN>
void bwd_un(const GraphView& g, float* dst, const float* P, int node_begin, int n_nodes,
            double* part, hipStream_t s) {
  const int tiles = (int)((g.T + kTile * UN - 1) / (kTile * UN));
  dim3 grid((unsigned)tiles, (unsigned)n_nodes);
  if (g.vec4)
    pointwise_bwd_kernel<TYPE, true, UN><<<grid, kBlock, 0, s>>>(g, dst, P, node_begin, part,
                                                                 tiles);
  else
    pointwise_bwd_kernel<TYPE, false, UN><<<grid, kBlock, 0, s>>>(g, dst, P, node_begin, part,
                                                                  tiles);
}

template <int TYPE>
hipError_t launch_bwd_t(const GraphView& g, float* dst, const float* P, int node_begin,
                        int n_nodes, double* part, hipStream_t s) {
  switch (g.pw_unroll) {
    case 2: bwd_un<TYPE, 2>(g, dst, P, node_begin, n_nodes, part, s); break;
    case 4: bwd_un<TYPE, 4>(g, dst, P, node_begin, n_nodes, part, s); break;
    default: bwd_un<TYPE, 1>(g, dst, P, node_begin, n_nodes, part, s); break;
  }
  return hipGetLastError();
}

}  // namespace

int pointwise_tiles(int64_t T, int unroll) {
  const int64_t tile = (int64_t)kTile * (unroll > 0 ? unroll : 1);
  return (int)((T + tile - 1) / tile);
}

hipError_t launch_pointwise_fwd(int type, const GraphView& g, float* U, const float* P,
                                int node_begin, int n_nodes, hipStream_t s) {
  switch (type) {
    case GRAFX_MIX:
    case GRAFX_OUT: return launch_fwd_t<GRAFX_MIX>(g, U, P, node_begin, n_nodes, s);
    case GRAFX_GAIN_PAN: return launch_fwd_t<GRAFX_GAIN_PAN>(g, U, P, node_begin, n_nodes, s);
    case GRAFX_IMAGER: return launch_fwd_t<GRAFX_IMAGER>(g, U, P, node_begin, n_nodes, s);
    case GRAFX_TANH: return launch_fwd_t<GRAFX_TANH>(g, U, P, node_begin, n_nodes, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pointwise_bwd(int type, const GraphView& g, float* dst, const float* P,
                                int node_begin, int n_nodes, double* part, hipStream_t s) {
  switch (type) {
    case GRAFX_IN:
    case GRAFX_MIX: return launch_bwd_t<GRAFX_MIX>(g, dst, P, node_begin, n_nodes, part, s);
    case GRAFX_GAIN_PAN: return launch_bwd_t<GRAFX_GAIN_PAN>(g, dst, P, node_begin, n_nodes, part, s);
    case GRAFX_IMAGER: return launch_bwd_t<GRAFX_IMAGER>(g, dst, P, node_begin, n_nodes, part, s);
    case GRAFX_TANH: return launch_bwd_t<GRAFX_TANH>(g, dst, P, node_begin, n_nodes, part, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce_partials(const ReduceJobs& jobs, hipStream_t s) {
  int blocks = 0;
  for (int q = 0; q < jobs.n; ++q) blocks += jobs.slots[q];
  if (blocks <= 0) return hipSuccess;
  reduce_partials_kernel<<<blocks, kBlock, 0, s>>>(jobs);
  return hipGetLastError();
}

}  // namespace grafx
