// Learned parameter initialiser for the gradient-descent mixing application (paper Sec. 4,
// "Example usage"): a convolutional encoder maps the log-mel features of a dry track and of the
// target mix to the normalised parameters of the track's gain/pan -> EQ -> compressor chain.
//
// Network: six convolution layers (kernel 5, stride 2, zero padding 2, bias, ReLU), 256 -> 64
// channels then 64 -> 64, frames F -> ceil(F/2) per layer; the mean over the remaining frames;
// one linear head 64 -> 11 and a sigmoid. Weights are one flat float32 buffer:
// [W1 (64 x 256 x 5), b1 (64), W2 (64 x 64 x 5), b2, ..., W6, b6, Wh (11 x 64), bh (11)].
//
// Training runs in float32 through hand-written kernels: forward, the mean-squared-error loss
// against the normalised labels, the backward of every layer (input gradients and weight
// gradients, each a fixed-order sum, so runs are bit-reproducible), and Adam. Inference can run
// the convolutions on the matrix cores: v_mfma_f32_16x16x16_bf16 with float32 accumulation, the
// layer as an implicit GEMM (M = 64 output channels, N = batch x frames, K = input channels x 5,
// the input window gathered per lane, no im2col buffer).
#include <cmath>

#include "device_common.h"
#include "grafx_internal.h"
#include "kernels.h"

namespace grafx {
namespace {

constexpr int kCin = 256, kCh = 64, kLayers = 6, kKs = 5, kOut = 11;

int frames_after(int f) { return (f + 1) / 2; }

struct EncLayout {
  int B, F[kLayers + 1];
  size_t w[kLayers + 2], b[kLayers + 2];  // weight and bias offsets (layer 1..6, head = 7)
  size_t n_w;
  size_t y[kLayers + 1], h, act;          // activations: y_l [B][64][F_l], pooled h [B][64]
  size_t dy[kLayers + 1], dh, dz, lossp, grad;  // backward scratch
};

int cin_of(int l) { return l == 1 ? kCin : kCh; }

EncLayout enc_layout(int B, int F) {
  EncLayout L{};
  L.B = B;
  L.F[0] = F;
  size_t o = 0;
  for (int l = 1; l <= kLayers; ++l) {
    L.F[l] = frames_after(L.F[l - 1]);
    L.w[l] = o;
    o += (size_t)kCh * cin_of(l) * kKs;
    L.b[l] = o;
    o += kCh;
  }
  L.w[kLayers + 1] = o;
  o += (size_t)kOut * kCh;
  L.b[kLayers + 1] = o;
  o += kOut;
  L.n_w = o;
  size_t a = 0, d = 0;
  for (int l = 1; l <= kLayers; ++l) {
    L.y[l] = a;
    a += (size_t)B * kCh * L.F[l];
    L.dy[l] = d;
    d += (size_t)B * kCh * L.F[l];
  }
  L.h = a;
  a += (size_t)B * kCh;
  L.act = a;
  L.dh = d;
  d += (size_t)B * kCh;
  L.dz = d;
  d += (size_t)B * kOut;
  L.lossp = d;
  d += (size_t)B;
  L.grad = d;
  return L;
}

// ---- float32 layers ---------------------------------------------------------------------------

// y[b][co][t] = ReLU(bias[co] + sum_{ci,k} W[co][ci][k] x[b][ci][2t + k - 2])
__global__ __launch_bounds__(kBlock) void conv_fwd_kernel(int B, int Cin, int Fin, int Fout,
                                                          const float* x, const float* W,
                                                          const float* bias, float* y) {
  const int64_t n = (int64_t)B * kCh * Fout;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * kBlock) {
    const int t = (int)(idx % Fout), co = (int)((idx / Fout) % kCh), b = (int)(idx / Fout / kCh);
    float acc = bias[co];
    const float* xb = x + (int64_t)b * Cin * Fin;
    const float* wc = W + (int64_t)co * Cin * kKs;
    for (int ci = 0; ci < Cin; ++ci)
#pragma unroll
      for (int k = 0; k < kKs; ++k) {
        const int src = 2 * t + k - 2;
        if (src >= 0 && src < Fin) acc = fmaf(wc[ci * kKs + k], xb[(int64_t)ci * Fin + src], acc);
      }
    y[idx] = fmaxf(acc, 0.f);
  }
}

// Mean over frames, the linear head and the sigmoid: one block of 64 threads per sample.
__global__ __launch_bounds__(64) void pool_head_kernel(int F6, const float* y6, const float* Wh,
                                                       const float* bh, float* h, float* s) {
  __shared__ float hs[kCh];
  const int b = blockIdx.x, c = threadIdx.x;
  float acc = 0.f;
  for (int t = 0; t < F6; ++t) acc += y6[((int64_t)b * kCh + c) * F6 + t];
  acc /= (float)F6;
  hs[c] = acc;
  h[(int64_t)b * kCh + c] = acc;
  __syncthreads();
  if (c < kOut) {
    float z = bh[c];
    for (int i = 0; i < kCh; ++i) z = fmaf(Wh[c * kCh + i], hs[i], z);
    s[(int64_t)b * kOut + c] = 1.f / (1.f + expf(-z));
  }
}

// Loss terms and the head's backward for one sample: dz = 2 (s - y) s (1 - s) / (B 11),
// dh = Wh^T dz, and the gradient of the pooled frames dy6[b][c][t] = dh[c] / F6.
__global__ __launch_bounds__(64) void head_bwd_kernel(int B, int F6, const float* s,
                                                      const float* labels, const float* Wh,
                                                      float* dz, float* dy6, float* lossp) {
  __shared__ float dzs[kOut], sq[kOut];
  const int b = blockIdx.x, c = threadIdx.x;
  if (c < kOut) {
    const float sv = s[(int64_t)b * kOut + c], d = sv - labels[(int64_t)b * kOut + c];
    const float g = 2.f * d / (float)(B * kOut) * sv * (1.f - sv);
    dzs[c] = g;
    sq[c] = d * d;
    dz[(int64_t)b * kOut + c] = g;
  }
  __syncthreads();
  float dh = 0.f;
  for (int o = 0; o < kOut; ++o) dh = fmaf(Wh[o * kCh + c], dzs[o], dh);
  for (int t = 0; t < F6; ++t) dy6[((int64_t)b * kCh + c) * F6 + t] = dh / (float)F6;
  if (c == 0) {
    float a = 0.f;
    for (int o = 0; o < kOut; ++o) a += sq[o];
    lossp[b] = a;
  }
}

// Head weight gradients (fixed order over the batch) and the loss value.
__global__ __launch_bounds__(kBlock) void head_grad_kernel(int B, const float* dz, const float* h,
                                                           const float* lossp, float* dWh,
                                                           float* dbh, float* loss) {
  for (int i = threadIdx.x; i < kOut * (kCh + 1); i += kBlock) {
    const int o = i / (kCh + 1), c = i % (kCh + 1);
    float acc = 0.f;
    for (int b = 0; b < B; ++b)
      acc = fmaf(dz[(int64_t)b * kOut + o], c < kCh ? h[(int64_t)b * kCh + c] : 1.f, acc);
    if (c < kCh)
      dWh[o * kCh + c] = acc;
    else
      dbh[o] = acc;
  }
  if (threadIdx.x == 0 && loss) {
    float a = 0.f;
    for (int b = 0; b < B; ++b) a += lossp[b];
    *loss = a / (float)(B * kOut);
  }
}

// dx[b][ci][f] = sum_{co,k: f = 2t + k - 2} W[co][ci][k] g[b][co][t], g = dy where y > 0.
__global__ __launch_bounds__(kBlock) void conv_bwd_data_kernel(int B, int Cin, int Fin, int Fout,
                                                               const float* W, const float* y,
                                                               const float* dy, float* dx) {
  const int64_t n = (int64_t)B * Cin * Fin;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * kBlock) {
    const int f = (int)(idx % Fin), ci = (int)((idx / Fin) % Cin), b = (int)(idx / Fin / Cin);
    float acc = 0.f;
    for (int co = 0; co < kCh; ++co) {
      const int64_t row = ((int64_t)b * kCh + co) * Fout;
#pragma unroll
      for (int k = 0; k < kKs; ++k) {
        const int t2 = f + 2 - k;
        if (t2 < 0 || (t2 & 1)) continue;
        const int t = t2 >> 1;
        if (t >= Fout) continue;
        const float g = y[row + t] > 0.f ? dy[row + t] : 0.f;
        acc = fmaf(W[((int64_t)co * Cin + ci) * kKs + k], g, acc);
      }
    }
    dx[idx] = acc;
  }
}

// dW[co][ci][k] = sum_{b,t} g[b][co][t] x[b][ci][2t + k - 2]: one block per (co, ci) for the
// five taps (blocks with ci = Cin give the bias gradient sum_{b,t} g); threads stride over
// (b, t) and a fixed-order block sum combines them.
__global__ __launch_bounds__(kBlock) void conv_bwd_weight_kernel(int B, int Cin, int Fin,
                                                                 int Fout, const float* x,
                                                                 const float* y, const float* dy,
                                                                 float* dW, float* db) {
  __shared__ float red[4];
  const int co = blockIdx.x % kCh, ci = blockIdx.x / kCh;
  float acc[kKs] = {0.f, 0.f, 0.f, 0.f, 0.f};
  const int n = B * Fout;
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const int b = i / Fout, t = i % Fout;
    const int64_t row = ((int64_t)b * kCh + co) * Fout;
    const float g = y[row + t] > 0.f ? dy[row + t] : 0.f;
    if (ci == Cin) {
      acc[0] += g;
      continue;
    }
    const float* xr = x + ((int64_t)b * Cin + ci) * Fin;
#pragma unroll
    for (int k = 0; k < kKs; ++k) {
      const int src = 2 * t + k - 2;
      if (src >= 0 && src < Fin) acc[k] = fmaf(g, xr[src], acc[k]);
    }
  }
  const int nk = ci == Cin ? 1 : kKs;
  for (int k = 0; k < nk; ++k) {
    const float v = block_sum<float>(acc[k], red);
    if (threadIdx.x == 0) {
      if (ci == Cin)
        db[co] = v;
      else
        dW[((int64_t)co * Cin + ci) * kKs + k] = v;
    }
  }
}

__global__ __launch_bounds__(kBlock) void adam_kernel(int64_t n, float* p, const float* g,
                                                      float* m, float* v, const float* scale,
                                                      float lr, float b1, float b2, float c1,
                                                      float c2, float eps) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= (scale ? lr * scale[i] : lr) * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// x[b] = [dry_feats[dry[b]]; mix_feats[mix[b]]] ([256][F]); labels[b] = label_table[dry[b]].
__global__ __launch_bounds__(kBlock) void gather_kernel(int B, int F, const float* dry_feats,
                                                        const int32_t* dry,
                                                        const float* mix_feats,
                                                        const int32_t* mix,
                                                        const float* label_table, float* labels,
                                                        float* x) {
  const int64_t n = (int64_t)B * kCin * F;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const int f = (int)(i % F), c = (int)((i / F) % kCin), b = (int)(i / F / kCin);
    const bool is_dry = c < kCin / 2;
    const float* table = is_dry ? dry_feats : mix_feats;
    const int src = is_dry ? dry[b] : mix[b];
    x[i] = table[((int64_t)src * (kCin / 2) + (c % (kCin / 2))) * F + f];
  }
  if (label_table)
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)B * kOut;
         i += (int64_t)gridDim.x * kBlock)
      labels[i] = label_table[(int64_t)dry[i / kOut] * kOut + i % kOut];
}

// Normalised outputs -> the chain's parameter rows: gain/pan dB [-12, 6] per channel, six EQ
// band gains [-12, 12] dB spread over 1024 log-magnitudes (linear in log-frequency between band
// centres 20 * 1000^((b + 0.5) / 6) Hz, bin k at k fs / 2047 Hz, constant beyond the outer
// centres), compressor time constant [1, 100] ms, threshold [-30, -10] dB, ratio [2, 8], knee
// 3 dB.
__global__ __launch_bounds__(kBlock) void params_kernel(const float* s, float* gp, float* eq,
                                                        float* comp) {
  const int b = blockIdx.x;
  const float* sb = s + (int64_t)b * kOut;
  const float ln10_20 = 0.11512925464970229f, ln10_10 = 0.23025850929940458f;
  __shared__ float band[6], lc[6];
  if (threadIdx.x < 6) {
    band[threadIdx.x] = -12.f + 24.f * sb[2 + threadIdx.x];
    lc[threadIdx.x] = logf(20.f) + logf(1000.f) * ((float)threadIdx.x + 0.5f) / 6.f;
  }
  if (threadIdx.x < 2) gp[(int64_t)b * 2 + threadIdx.x] = (-12.f + 18.f * sb[threadIdx.x]) * ln10_20;
  if (threadIdx.x == 0) {
    const float tau = 1.f + 99.f * sb[8];
    comp[(int64_t)b * 4 + 0] = expf(-1.f / (tau * 1e-3f * 44100.f));
    comp[(int64_t)b * 4 + 1] = (-30.f + 20.f * sb[9]) * ln10_10;
    comp[(int64_t)b * 4 + 2] = 3.f * ln10_10;
    comp[(int64_t)b * 4 + 3] = 2.f + 6.f * sb[10];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 1024; k += kBlock) {
    const float lf = logf(fmaxf((float)k * 44100.f / 2047.f, 1e-3f));
    float gdb;
    if (lf <= lc[0]) {
      gdb = band[0];
    } else if (lf >= lc[5]) {
      gdb = band[5];
    } else {
      int i = 0;
      while (lf >= lc[i + 1]) ++i;
      gdb = band[i] + (band[i + 1] - band[i]) * (lf - lc[i]) / (lc[i + 1] - lc[i]);
    }
    eq[(int64_t)b * 1024 + k] = gdb * ln10_20;
  }
}

// ---- bfloat16 matrix-core convolution (inference) ----------------------------------------------

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {  // round to nearest even
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// A block computes all 64 output channels over 64 columns n = b * Fout + t. The K dimension
// (in channel x tap, K = Cin * 5) advances in chunks of 128: the block stages the weight chunk
// A[64][128] and the gathered input chunk Bt[64 columns][128] in LDS as bfloat16 (nearest even),
// then wave w multiplies rows 16 w .. 16 w + 15 against the four 16-column tiles, eight K steps
// of v_mfma_f32_16x16x16_bf16 each. Large chunks amortise the global-load latency of staging,
// which bounds the kernel at these sizes. Operands per lane l = i + 16 q: A row i, K entries 4q..4q+3;
// B column i, K entries 4q..4q+3; D column i, rows 4q..4q+3. Rows of the LDS tiles are padded
// by 4 bf16 so the 16 lanes of a fragment read distinct banks.
constexpr int kMN = 64, kKC = 128, kLd = kKC + 4;
constexpr int kStage = kKC / 4;  // K entries staged per thread and chunk

__global__ __launch_bounds__(kBlock) void conv_fwd_mfma_kernel(int B, int Cin, int Fin, int Fout,
                                                               const float* x, const float* W,
                                                               const float* bias, float* y) {
  __shared__ short As[kMN * kLd], Bs[kMN * kLd];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 15, q = lane >> 4;
  const int N = B * Fout, K = Cin * kKs;
  const int n0 = blockIdx.x * kMN;
  // staging roles. A: thread r covers channel r / 4 and the kStage consecutive K entries
  // kStage (r % 4) .. (contiguous weights). B: thread r covers column r % 64 and the K entries
  // kStage (r / 64) .., so a wave reads 64 neighbouring columns (frames two samples apart) at
  // every K entry.
  const int srow = threadIdx.x >> 2, sk = (threadIdx.x & 3) * kStage;
  const int bn = threadIdx.x & 63, bk = (threadIdx.x >> 6) * kStage;
  const int n_s = n0 + bn;
  const bool live_s = n_s < N;
  const int b_s = live_s ? n_s / Fout : 0, t_s = live_s ? n_s % Fout : 0;
  // one wave-uniform descriptor per tensor (per-lane descriptors would make the compiler loop
  // over the lanes for every load); the host keeps both tensors below 2^29 elements
  const auto rx = row_rsrc(x, (int64_t)B * Cin * Fin);
  const auto rw = row_rsrc(W, (int64_t)kCh * K);
  const int xbase = b_s * Cin * Fin, wbase = srow * K;
  f32x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += kKC) {
    __syncthreads();  // the previous chunk's fragments have been read
    float va[kStage], vb[kStage];  // every load of the chunk in flight before any is used
#pragma unroll
    for (int e = 0; e < kStage; ++e) {  // branch-free: out-of-range offsets read 0 in hardware
      const int ka = k0 + sk + e;
      va[e] = bload(rw, ka < K ? wbase + ka : -1);
      const int kb = k0 + bk + e;
      const int ci = kb / kKs, tap = kb % kKs;
      const int src = 2 * t_s + tap - 2;
      const bool ok = live_s && kb < K && src >= 0 && src < Fin;
      vb[e] = bload(rx, ok ? xbase + ci * Fin + src : -1);
    }
#pragma unroll
    for (int e = 0; e < kStage; ++e) {
      As[srow * kLd + sk + e] = to_bf16(va[e]);
      Bs[bn * kLd + bk + e] = to_bf16(vb[e]);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kKC; ks += 16) {
      bf16x4 a;
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = As[(wave * 16 + i) * kLd + ks + 4 * q + e];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bf16x4 bv;
#pragma unroll
        for (int e = 0; e < 4; ++e) bv[e] = Bs[(j * 16 + i) * kLd + ks + 4 * q + e];
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[j], 0, 0, 0);
      }
    }
  }
  float bsum[4];  // this lane's four channels, loaded once before the stores
#pragma unroll
  for (int e = 0; e < 4; ++e) bsum[e] = bias[wave * 16 + 4 * q + e];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + j * 16 + i;
    if (n >= N) continue;
    const int b = n / Fout, t = n % Fout;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int co = wave * 16 + 4 * q + e;
      y[((int64_t)b * kCh + co) * Fout + t] = fmaxf(acc[j][e] + bsum[e], 0.f);
    }
  }
}

unsigned grid_for(int64_t n) {
  const int64_t g = (n + kBlock - 1) / kBlock;
  return (unsigned)(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

grafx_status hip_st(hipError_t e, const char* what) {
  if (e == hipSuccess) return GRAFX_OK;
  return fail(GRAFX_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

grafx_status check_dims(int32_t batch, int32_t frames) {
  if (batch < 1 || batch > (1 << 20)) return fail(GRAFX_E_SHAPE, "batch must be in [1, 2^20]");
  if (frames < 1 || frames > (1 << 20)) return fail(GRAFX_E_SHAPE, "frames must be in [1, 2^20]");
  return GRAFX_OK;
}

}  // namespace
}  // namespace grafx

using namespace grafx;

extern "C" {

grafx_status grafx_encoder_sizes(int32_t batch, int32_t frames, size_t* n_weights,
                                 size_t* act_floats, size_t* grad_floats) {
  clear_error();
  grafx_status st = check_dims(batch, frames);
  if (st != GRAFX_OK) return st;
  const EncLayout L = enc_layout(batch, frames);
  if (n_weights) *n_weights = L.n_w;
  if (act_floats) *act_floats = L.act;
  if (grad_floats) *grad_floats = L.grad;
  return GRAFX_OK;
}

grafx_status grafx_logmel(int32_t n_signals, int64_t T, const float* signals, float* features,
                          hipStream_t stream) {
  clear_error();
  if (n_signals < 1) return fail(GRAFX_E_SHAPE, "n_signals must be >= 1");
  if (T < 1024 || T >= ((int64_t)1 << 29)) return fail(GRAFX_E_SHAPE, "T must be in [1024, 2^29)");
  if (!signals || !features) return fail(GRAFX_E_ARG, "NULL argument");
  return hip_st(launch_logmel(n_signals, T, signals, features, stream), "logmel launch");
}

grafx_status grafx_encoder_gather(int32_t batch, int32_t frames, const float* dry_features,
                                  const int32_t* dry, const float* mix_features,
                                  const int32_t* mix, const float* label_table, float* labels,
                                  float* x, hipStream_t stream) {
  clear_error();
  grafx_status st = check_dims(batch, frames);
  if (st != GRAFX_OK) return st;
  if (!dry_features || !dry || !mix_features || !mix || !x || (label_table && !labels))
    return fail(GRAFX_E_ARG, "NULL argument");
  const int64_t n = (int64_t)batch * kCin * frames;
  gather_kernel<<<grid_for(n), kBlock, 0, stream>>>(batch, frames, dry_features, dry,
                                                    mix_features, mix, label_table, labels, x);
  return hip_st(hipGetLastError(), "encoder_gather launch");
}

grafx_status grafx_encoder_forward(int32_t batch, int32_t frames, const float* x,
                                   const float* weights, int32_t bf16, float* acts, float* out,
                                   hipStream_t stream) {
  clear_error();
  grafx_status st = check_dims(batch, frames);
  if (st != GRAFX_OK) return st;
  if (!x || !weights || !acts || !out) return fail(GRAFX_E_ARG, "NULL argument");
  if (bf16 && (int64_t)batch * kCin * frames >= ((int64_t)1 << 29))
    return fail(GRAFX_E_SHAPE, "bf16 forward: batch x 256 x frames must be below 2^29");
  const EncLayout L = enc_layout(batch, frames);
  const float* in = x;
  hipError_t e = hipSuccess;
  for (int l = 1; l <= kLayers && e == hipSuccess; ++l) {
    float* y = acts + L.y[l];
    const int Cin = cin_of(l);
    if (bf16) {
      const int cols = batch * L.F[l];
      conv_fwd_mfma_kernel<<<(cols + kMN - 1) / kMN, kBlock, 0, stream>>>(
          batch, Cin, L.F[l - 1], L.F[l], in, weights + L.w[l], weights + L.b[l], y);
    } else {
      const int64_t n = (int64_t)batch * kCh * L.F[l];
      conv_fwd_kernel<<<grid_for(n), kBlock, 0, stream>>>(batch, Cin, L.F[l - 1], L.F[l], in,
                                                          weights + L.w[l], weights + L.b[l], y);
    }
    e = hipGetLastError();
    in = y;
  }
  if (e == hipSuccess) {
    pool_head_kernel<<<batch, 64, 0, stream>>>(L.F[kLayers], acts + L.y[kLayers],
                                               weights + L.w[kLayers + 1],
                                               weights + L.b[kLayers + 1], acts + L.h, out);
    e = hipGetLastError();
  }
  return hip_st(e, "encoder_forward launch");
}

grafx_status grafx_encoder_backward(int32_t batch, int32_t frames, const float* x,
                                    const float* weights, const float* acts, const float* out,
                                    const float* labels, float* loss, float* dweights,
                                    float* grads, hipStream_t stream) {
  clear_error();
  grafx_status st = check_dims(batch, frames);
  if (st != GRAFX_OK) return st;
  if (!x || !weights || !acts || !out || !labels || !dweights || !grads)
    return fail(GRAFX_E_ARG, "NULL argument");
  const EncLayout L = enc_layout(batch, frames);
  head_bwd_kernel<<<batch, 64, 0, stream>>>(batch, L.F[kLayers], out, labels,
                                            weights + L.w[kLayers + 1], grads + L.dz,
                                            grads + L.dy[kLayers], grads + L.lossp);
  head_grad_kernel<<<1, kBlock, 0, stream>>>(batch, grads + L.dz, acts + L.h, grads + L.lossp,
                                             dweights + L.w[kLayers + 1],
                                             dweights + L.b[kLayers + 1], loss);
  hipError_t e = hipGetLastError();
  for (int l = kLayers; l >= 1 && e == hipSuccess; --l) {
    const int Cin = cin_of(l);
    const float* xin = l == 1 ? x : acts + L.y[l - 1];
    const float* y = acts + L.y[l];
    const float* dy = grads + L.dy[l];
    conv_bwd_weight_kernel<<<kCh * (Cin + 1), kBlock, 0, stream>>>(
        batch, Cin, L.F[l - 1], L.F[l], xin, y, dy, dweights + L.w[l], dweights + L.b[l]);
    if (l > 1) {
      const int64_t n = (int64_t)batch * Cin * L.F[l - 1];
      conv_bwd_data_kernel<<<grid_for(n), kBlock, 0, stream>>>(
          batch, Cin, L.F[l - 1], L.F[l], weights + L.w[l], y, dy, grads + L.dy[l - 1]);
    }
    e = hipGetLastError();
  }
  return hip_st(e, "encoder_backward launch");
}

grafx_status grafx_adam(int64_t n, float* p, const float* g, float* m, float* v,
                        const float* lr_scale, int32_t step, float lr, float beta1, float beta2,
                        float eps, hipStream_t stream) {
  clear_error();
  if (n < 0 || step < 1) return fail(GRAFX_E_ARG, "n must be >= 0 and step >= 1");
  if (n == 0) return GRAFX_OK;
  if (!p || !g || !m || !v) return fail(GRAFX_E_ARG, "NULL argument");
  const float c1 = (float)(1.0 - std::pow((double)beta1, step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, step));
  adam_kernel<<<grid_for(n), kBlock, 0, stream>>>(n, p, g, m, v, lr_scale, lr, beta1, beta2, c1,
                                                  c2, eps);
  return hip_st(hipGetLastError(), "adam launch");
}

grafx_status grafx_encoder_params(int32_t batch, const float* out, float* gain_pan, float* eq,
                                  float* comp, hipStream_t stream) {
  clear_error();
  if (batch < 1) return fail(GRAFX_E_SHAPE, "batch must be >= 1");
  if (!out || !gain_pan || !eq || !comp) return fail(GRAFX_E_ARG, "NULL argument");
  params_kernel<<<batch, kBlock, 0, stream>>>(out, gain_pan, eq, comp);
  return hip_st(hipGetLastError(), "encoder_params launch");
}

}  // extern "C"
