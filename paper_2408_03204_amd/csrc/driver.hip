// Render drivers: the host step loops of the batched render (paper Algorithm 1, main loop) and
// of its adjoint, the plan upload and the workspace layout. Every argument is checked before the
// first launch; the drivers only enqueue kernels on the caller's stream.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "device_common.h"
#include "grafx_internal.h"
#include "kernels.h"

// Workspace of grafx_render_noalloc: a file-scope device array, one copy per GPU, held until the
// process ends. In host code its name is not a device address: the address comes from
// hipGetSymbolAddress, looked up once per device (with that device current) by noalloc_scratch.
static constexpr size_t kNoallocScratchBytes = GRAFX_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace grafx {
namespace {

// Workspace layout (byte offsets, 256-byte aligned sections). The forward part is kept by the
// render for the adjoint: EQ filters, dynamics carries, delay taps. "Dynamics" rows are the
// compressor nodes (by parameter slot) followed by the noisegate nodes: both run the same
// envelope scan and share one set of chunk totals, carries, tickets and gradient partials.
struct WsLayout {
  size_t eq_h, eq_H, comp_agg, comp_carry, comp_tickets, delay_taps[2], delay_offs[2];
  size_t ar_slots, ar_carry, ar_pat, ar_tickets;
  size_t rv_Un, rv_h, rv_H, rv_Z, rv_C;
  size_t fwd_end;
  size_t part_gp, part_im, part_tanh, comp_ragg, comp_part, eq_C, eq_spec, eq_s, delay_part[2];
  size_t ar_ragg, ar_part;
  size_t rv_Y0, rv_G, rv_hbar, rv_part, rv_len;
  size_t dl_X[2], dl_Y0[2], dl_G[2], dl_R[2], dl_len[2];
  size_t total;
};

// Dynamics rows: compressors first, then noisegates.
size_t n_dynamics(const grafx_schedule_t* h) {
  return (size_t)h->type_count[GRAFX_COMPRESSOR] + h->type_count[GRAFX_NOISEGATE];
}
int dyn_row(const grafx_schedule_t* h, int t) {
  return t == GRAFX_NOISEGATE ? h->type_count[GRAFX_COMPRESSOR] : 0;
}

// The two multitap delay types (family 0: 500 ms, 5 slots; family 1: 2 s, 20 slots) run the same
// kernels and keep separate workspace sections.
constexpr int kDelayType[2] = {GRAFX_DELAY, GRAFX_DELAY_LONG};
constexpr int kDelaySlots[2] = {kDelayTaps, kDelayTapsLong};
int delay_family(int t) { return t == GRAFX_DELAY_LONG ? 1 : 0; }

// Published words per attack/release node: kArPasses pass rows of (A, B, flag), then the final
// (A, B) of every chunk.
size_t ar_slot_words(size_t chunks) { return (size_t)kArPasses * chunks * 3 + chunks * 2; }

WsLayout ws_layout(const grafx_schedule_t* h, int64_t T, bool with_bwd) {
  WsLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  const size_t n_eq = h->type_count[GRAFX_EQ];
  const size_t n_comp = n_dynamics(h);
  const size_t chunks = comp_chunks(T);
  L.eq_h = take(n_eq * 1024 * sizeof(double));
  L.eq_H = take(n_eq * kEqFFT * sizeof(float));
  L.comp_agg = take(n_comp * chunks * sizeof(uint64_t));
  L.comp_carry = take(n_comp * chunks * sizeof(double));
  // the error word on a cache line of its own, then one ticket counter per dynamics node
  // (forward) and one per node (adjoint), each on its own cache line
  L.comp_tickets = take((1 + 2 * n_comp) * kCompTicketStride * sizeof(unsigned));
  for (int f = 0; f < 2; ++f) {
    const size_t n_del = h->type_count[kDelayType[f]];
    L.delay_taps[f] = take(n_del * delay_coef(kDelaySlots[f]) * sizeof(float));
    L.delay_offs[f] = take(n_del * 2 * kDelaySlots[f] * sizeof(int32_t));
  }
  // attack/release compressors: per-pass and final chunk maps (reset), entering states and final
  // branch patterns (kept for the adjoint), forward then adjoint ticket counters
  const size_t n_ar = h->type_count[GRAFX_COMPRESSOR_AR];
  L.ar_slots = take(n_ar * ar_slot_words(chunks) * sizeof(uint64_t));
  L.ar_carry = take(n_ar * chunks * sizeof(double));
  L.ar_pat = take(n_ar * chunks * kBlock * sizeof(uint16_t));
  L.ar_tickets = take(2 * n_ar * kCompTicketStride * sizeof(unsigned));
  // reverb: noise STFT (shared), FIRs, partition spectra, input-window spectra (kept for the
  // FIR gradient)
  const size_t n_rv = h->type_count[GRAFX_REVERB];
  const size_t rv_L = n_rv ? (size_t)h->rv_len : 0;
  const size_t rv_M = n_rv ? (size_t)rv_frames(h->rv_len) : 0;
  const size_t rv_P = n_rv ? (size_t)rv_parts(h->rv_len) : 0;
  const size_t rv_nb = n_rv ? (size_t)rv_blocks(T) : 0;
  L.rv_Un = take(2 * rv_M * (kRvFft / 2 + 1) * sizeof(double2));
  L.rv_h = take(n_rv * 2 * rv_L * sizeof(float));
  L.rv_H = take(n_rv * rv_P * kRvStride * sizeof(float4));
  L.rv_Z = take(n_rv * rv_nb * kRvStride * sizeof(float4));
  L.rv_C = take(n_rv * (n_rv ? (size_t)rv_conv_tiles(h->rv_len) : 0) * rv_nb * kRvStride *
                sizeof(float4));
  L.fwd_end = off;
  if (with_bwd) {
    const size_t tiles = pointwise_tiles(T);
    L.part_gp = take(h->type_count[GRAFX_GAIN_PAN] * tiles * 2 * sizeof(double));
    L.part_im = take(h->type_count[GRAFX_IMAGER] * tiles * sizeof(double));
    L.part_tanh = take(h->type_count[GRAFX_TANH] * tiles * sizeof(double));
    L.comp_ragg = take(n_comp * chunks * sizeof(uint64_t));
    L.comp_part = take(n_comp * chunks * 4 * sizeof(double));
    // EQ adjoint partials: a region per EQ node (parameter row), summed once after the last step
    L.eq_C = take(n_eq * (size_t)eq_tiles(T) * kEqFoldStride * sizeof(float));
    L.eq_spec = take(n_eq * kEqFoldStride * sizeof(float));
    L.eq_s = take(n_eq * 1024 * sizeof(double));
    // sized for the smallest tap-gradient group, so that the size does not depend on tuning
    for (int f = 0; f < 2; ++f)
      L.delay_part[f] = take((size_t)h->type_count[kDelayType[f]] * delay_groups(T, kTapTilesMin) *
                             delay_coef(kDelaySlots[f]) * sizeof(float));
    L.ar_ragg = take(n_ar * chunks * 2 * sizeof(uint64_t));
    L.ar_part = take(n_ar * chunks * kArParams * sizeof(double));
    L.rv_Y0 = take(n_rv * rv_nb * kRvStride * sizeof(float4));
    L.rv_G = take(n_rv * rv_P * kRvStride * sizeof(float4));
    L.rv_hbar = take(n_rv * 2 * rv_L * sizeof(float));
    L.rv_part = take(n_rv * (n_rv ? (size_t)rv_grad_blocks(h->rv_len) : 0) * 2 *
                     (kRvFft / 2 + 1) * sizeof(double2));
    L.rv_len = take(n_rv * sizeof(int32_t));  // each reverb node's length, by slot
    // delay-time surrogate: input-window and adjoint-block spectra, cross-spectra, correlation
    for (int f = 0; f < 2; ++f) {
      const size_t n_sur = h->delay_surrogate ? (size_t)h->type_count[kDelayType[f]] : 0;
      const size_t sur_nb = n_sur ? (size_t)rv_blocks(T + kDelaySurShift) : 0;
      L.dl_X[f] = take(n_sur * sur_nb * kRvStride * sizeof(float4));
      L.dl_Y0[f] = take(n_sur * sur_nb * kRvStride * sizeof(float4));
      L.dl_G[f] = take(n_sur * delay_sur_parts(kDelaySlots[f]) * kRvStride * sizeof(float4));
      L.dl_R[f] = take(n_sur * 2 * delay_sur_len(kDelaySlots[f]) * sizeof(float));
      L.dl_len[f] = take(n_sur * sizeof(int32_t));
    }
  }
  L.total = off;
  return L;
}

template <typename P>
P* at(void* ws, size_t off) {
  return reinterpret_cast<P*>(static_cast<char*>(ws) + off);
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

GraphView make_view(const grafx_schedule_t* h, const void* dev_plan, int64_t T, const float* S,
                    const float* U) {
  const int32_t* plan = static_cast<const int32_t*>(dev_plan);
  GraphView g{};
  g.in_ptr = plan + h->layout.in_ptr;
  g.in_src = plan + h->layout.in_src;
  g.out_ptr = plan + h->layout.out_ptr;
  g.out_dst = plan + h->layout.out_dst;
  g.param_row = plan + h->layout.param_row;
  g.len = h->node_len.empty() ? nullptr : plan + h->layout.len;
  g.S = S;
  g.U = U;
  g.T = T;
  g.K = h->K;
  g.out_begin = h->step_ptr[h->N];
  g.vec4 = (T % 4 == 0) && h->len4;
  g.pw_unroll = h->pw_unroll;
  g.wait_polls = h->wait_polls;
  g.eq_order = h->eq_order;
  g.dyn_order = h->dyn_order;
  g.tap_tiles = h->tap_tiles;
  return g;
}

grafx_status check_common(const grafx_schedule_t* h, const void* dev_plan, int64_t T,
                          const float* S, const float* const* P, const float* U, void* ws,
                          size_t ws_bytes, bool with_bwd) {
  if (!h) return fail(GRAFX_E_ARG, "schedule is NULL");
  if (!dev_plan) return fail(GRAFX_E_ARG, "plan is NULL");
  if (T < 1) return fail(GRAFX_E_SHAPE, "T must be >= 1");
  if (h->max_len > T)
    return fail(GRAFX_E_SHAPE, "T (the row stride) is below the largest node length " +
                                   std::to_string(h->max_len));
  if (T >= ((int64_t)1 << 29)) return fail(GRAFX_E_SHAPE, "T must be < 2^29");
  if (!U) return fail(GRAFX_E_ARG, "U is NULL");
  if (h->K > 0 && !S) return fail(GRAFX_E_ARG, "S is NULL but the graph has input nodes");
  if (!aligned(dev_plan, 256)) return fail(GRAFX_E_SHAPE, "plan must be 256-byte aligned");
  if (!aligned(U, 16) || (S && !aligned(S, 16)))
    return fail(GRAFX_E_SHAPE, "signal buffers must be 16-byte aligned");
  for (int t = 0; t < kNumTypes; ++t)
    if (kParamCount[t] > 0 && h->type_count[t] > 0 && (!P || !P[t]))
      return fail(GRAFX_E_SHAPE, "missing parameter tensor for node type " + std::to_string(t));
  if (h->type_count[GRAFX_REVERB] > 0 && !h->rv_noise)
    return fail(GRAFX_E_ARG,
                "the graph has reverb nodes but no noise was set (grafx_schedule_set_reverb_noise)");
  const WsLayout L = ws_layout(h, T, with_bwd);
  if (L.total > 0 && (!ws || ws_bytes < L.total))
    return fail(GRAFX_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total) +
                                       " bytes, got " + std::to_string(ws_bytes));
  if (ws && !aligned(ws, 256)) return fail(GRAFX_E_SHAPE, "workspace must be 256-byte aligned");
  return GRAFX_OK;
}

unsigned* error_word(void* ws, const WsLayout& L) { return at<unsigned>(ws, L.comp_tickets); }

unsigned* tickets(void* ws, const WsLayout& L, const grafx_schedule_t* h, bool bwd) {
  return error_word(ws, L) +
         (size_t)(1 + (bwd ? n_dynamics(h) : 0)) * kCompTicketStride;
}

bool is_dynamics(int t) { return t == GRAFX_COMPRESSOR || t == GRAFX_NOISEGATE; }
bool has_dynamics(const grafx_schedule_t* h) {
  return n_dynamics(h) + h->type_count[GRAFX_COMPRESSOR_AR] > 0;
}

// Reset the dynamics chaining state of one pass (all compressor and noisegate nodes, all steps).
// The forward reset also clears the error word, which sits just before the forward tickets; it
// runs whenever the graph has any dynamics node (attack/release compressors included).
hipError_t reset_comp(const grafx_schedule_t* h, void* ws, const WsLayout& L, bool bwd,
                      int64_t T, hipStream_t stream) {
  const int n_comp = n_dynamics(h);
  if (!has_dynamics(h) || (bwd && n_comp == 0)) return hipSuccess;
  uint64_t* tot = at<uint64_t>(ws, bwd ? L.comp_ragg : L.comp_agg);
  if (bwd)
    return launch_comp_reset(tot, (int64_t)n_comp * comp_chunks(T), tickets(ws, L, h, true),
                             n_comp * kCompTicketStride, stream);
  return launch_comp_reset(tot, (int64_t)n_comp * comp_chunks(T), error_word(ws, L),
                           (1 + n_comp) * kCompTicketStride, stream);
}

// Reset the attack/release chaining state of one pass.
hipError_t reset_ar(const grafx_schedule_t* h, void* ws, const WsLayout& L, bool bwd, int64_t T,
                    hipStream_t stream) {
  const int n_ar = h->type_count[GRAFX_COMPRESSOR_AR];
  if (n_ar == 0) return hipSuccess;
  const size_t chunks = comp_chunks(T);
  unsigned* t = at<unsigned>(ws, L.ar_tickets) + (bwd ? (size_t)n_ar * kCompTicketStride : 0);
  if (bwd)
    return launch_comp_reset(at<uint64_t>(ws, L.ar_ragg), (int64_t)(n_ar * chunks * 2), t,
                             n_ar * kCompTicketStride, stream);
  return launch_comp_reset(at<uint64_t>(ws, L.ar_slots), (int64_t)(n_ar * ar_slot_words(chunks)),
                           t, n_ar * kCompTicketStride, stream);
}

// The dynamics block order of one launch: the setting, or for "auto" (2) interleaved nodes once a
// launch spans several rounds of resident blocks (then a chunk's predecessors have usually
// published by the time it starts) and a node's chunks together for about one round.
constexpr int kDynInterleaveBlocks = 4096;
GraphView dyn_view(const GraphView& g, int n_nodes) {
  GraphView d = g;
  if (d.dyn_order == 2) d.dyn_order = (int64_t)n_nodes * comp_chunks(g.T) >= kDynInterleaveBlocks;
  return d;
}

hipError_t enqueue_fwd_step(const grafx_schedule_t* h, const GraphView& g, const float* const* P,
                            float* U, void* ws, const WsLayout& L, int n, hipStream_t stream) {
  const int t = h->step_type[n];
  const int b = h->step_ptr[n], cnt = h->step_ptr[n + 1] - b;
  if (cnt == 0) return hipSuccess;
  const float* p = P ? P[t] : nullptr;
  switch (t) {
    case GRAFX_MIX:
    case GRAFX_OUT:
    case GRAFX_GAIN_PAN:
    case GRAFX_IMAGER:
    case GRAFX_TANH:
      return launch_pointwise_fwd(t, g, U, p, b, cnt, stream);
    case GRAFX_EQ:
      return launch_eq_fwd(g, U, at<float>(ws, L.eq_H), b, cnt, stream);
    case GRAFX_COMPRESSOR:
    case GRAFX_NOISEGATE:
      return launch_comp_fwd(dyn_view(g, cnt), U, p, b, cnt, dyn_row(h, t), t == GRAFX_NOISEGATE,
                             at<uint64_t>(ws, L.comp_agg),
                             at<double>(ws, L.comp_carry), tickets(ws, L, h, false),
                             error_word(ws, L), stream);
    case GRAFX_DELAY:
    case GRAFX_DELAY_LONG: {
      const int f = delay_family(t);
      return launch_delay_fwd(kDelaySlots[f], g, U, at<float>(ws, L.delay_taps[f]),
                              at<int32_t>(ws, L.delay_offs[f]), b, cnt, stream);
    }
    case GRAFX_COMPRESSOR_AR: {
      const size_t n_ar = h->type_count[GRAFX_COMPRESSOR_AR], chunks = comp_chunks(g.T);
      uint64_t* slots = at<uint64_t>(ws, L.ar_slots);
      return launch_comp_ar_fwd(dyn_view(g, cnt), U, p, b, cnt, h->ar_max_pass, slots,
                                slots + n_ar * (size_t)kArPasses * chunks * 3,
                                at<double>(ws, L.ar_carry), at<uint16_t>(ws, L.ar_pat),
                                at<unsigned>(ws, L.ar_tickets), error_word(ws, L), stream);
    }
    case GRAFX_REVERB:
      return launch_rv_fwd(g, U, b, cnt, h->rv_len, at<float4>(ws, L.rv_H), at<float4>(ws, L.rv_Z),
                           at<float4>(ws, L.rv_C), stream);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t enqueue_bwd_step(const grafx_schedule_t* h, const GraphView& g, const float* const* P,
                            float* dU, void* ws, const WsLayout& L, int n, hipStream_t stream) {
  const int t = h->step_type[n];
  const int b = h->step_ptr[n], cnt = h->step_ptr[n + 1] - b;
  if (cnt == 0) return hipSuccess;
  const float* p = P ? P[t] : nullptr;
  switch (t) {
    case GRAFX_MIX:
      return launch_pointwise_bwd(t, g, dU, nullptr, b, cnt, nullptr, stream);
    case GRAFX_GAIN_PAN:
      return launch_pointwise_bwd(t, g, dU, p, b, cnt, at<double>(ws, L.part_gp), stream);
    case GRAFX_IMAGER:
      return launch_pointwise_bwd(t, g, dU, p, b, cnt, at<double>(ws, L.part_im), stream);
    case GRAFX_TANH:
      return launch_pointwise_bwd(t, g, dU, p, b, cnt, at<double>(ws, L.part_tanh), stream);
    case GRAFX_EQ:
      return launch_eq_bwd(g, dU, at<float>(ws, L.eq_H), b, cnt, at<float>(ws, L.eq_C), stream);
    case GRAFX_COMPRESSOR:
    case GRAFX_NOISEGATE:
      return launch_comp_bwd(dyn_view(g, cnt), dU, p, b, cnt, dyn_row(h, t), t == GRAFX_NOISEGATE,
                             at<double>(ws, L.comp_carry),
                             at<uint64_t>(ws, L.comp_ragg), at<double>(ws, L.comp_part),
                             tickets(ws, L, h, true), error_word(ws, L), stream);
    case GRAFX_DELAY:
    case GRAFX_DELAY_LONG: {
      const int f = delay_family(t);
      hipError_t e = launch_delay_bwd(kDelaySlots[f], g, dU, at<float>(ws, L.delay_taps[f]),
                                      at<int32_t>(ws, L.delay_offs[f]), b, cnt,
                                      at<float>(ws, L.delay_part[f]), stream);
      // R[n] = sum_t ybar[t - 19] u[t - n]: lag n - 19 of the plain correlation
      const int nb = rv_blocks(g.T + kDelaySurShift);
      if (e == hipSuccess && h->delay_surrogate)
        e = launch_xcorr_spectra(g, b, cnt, false, 0, nb, at<float4>(ws, L.dl_X[f]), nullptr,
                                 stream);
      if (e == hipSuccess && h->delay_surrogate)
        e = launch_xcorr_spectra(g, b, cnt, true, -kDelaySurShift, nb, at<float4>(ws, L.dl_Y0[f]),
                                 at<int32_t>(ws, L.dl_len[f]), stream);
      return e;
    }
    case GRAFX_COMPRESSOR_AR:
      return launch_comp_ar_bwd(dyn_view(g, cnt), dU, p, b, cnt, at<double>(ws, L.ar_carry),
                                at<uint16_t>(ws, L.ar_pat), at<uint64_t>(ws, L.ar_ragg),
                                at<double>(ws, L.ar_part),
                                at<unsigned>(ws, L.ar_tickets) +
                                    (size_t)h->type_count[GRAFX_COMPRESSOR_AR] * kCompTicketStride,
                                error_word(ws, L), stream);
    case GRAFX_REVERB:
      return launch_rv_bwd(g, dU, b, cnt, h->rv_len, at<float4>(ws, L.rv_H),
                           at<float4>(ws, L.rv_Y0), at<float4>(ws, L.rv_C),
                           at<int32_t>(ws, L.rv_len), stream);
    default:
      return hipErrorInvalidValue;
  }
}

grafx_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return GRAFX_OK;
  return fail(GRAFX_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// The forward loop of grafx_render on a workspace that has passed the checks: per-render
// parameter preprocessing, reset of the dynamics chaining state, then steps 1..N.
grafx_status enqueue_render(const grafx_schedule_t* h, const void* dev_plan, int64_t T,
                            const float* S, const float* const* P, float* U, void* ws,
                            hipStream_t stream) {
  const WsLayout L = ws_layout(h, T, false);
  const GraphView g = make_view(h, dev_plan, T, S, U);
  auto par = [&](int t) -> const float* { return P ? P[t] : nullptr; };
  hipError_t e = hipSuccess;
  // per-render parameter preprocessing
  if (h->type_count[GRAFX_EQ] > 0)
    e = launch_eq_design(par(GRAFX_EQ), h->type_count[GRAFX_EQ], at<double>(ws, L.eq_h),
                         at<float>(ws, L.eq_H), stream);
  for (int f = 0; f < 2 && e == hipSuccess; ++f)
    if (h->type_count[kDelayType[f]] > 0)
      e = launch_delay_design(kDelaySlots[f], par(kDelayType[f]), h->type_count[kDelayType[f]],
                              at<float>(ws, L.delay_taps[f]), at<int32_t>(ws, L.delay_offs[f]),
                              stream);
  if (e == hipSuccess && h->type_count[GRAFX_REVERB] > 0)
    e = launch_rv_design(par(GRAFX_REVERB), h->type_count[GRAFX_REVERB], h->rv_noise, h->rv_len,
                         at<double2>(ws, L.rv_Un), at<float>(ws, L.rv_h), at<float4>(ws, L.rv_H),
                         stream);
  if (e == hipSuccess) e = reset_comp(h, ws, L, false, T, stream);
  if (e == hipSuccess) e = reset_ar(h, ws, L, false, T, stream);
  for (int n = 1; n <= h->N && e == hipSuccess; ++n)
    e = enqueue_fwd_step(h, g, P, U, ws, L, n, stream);
  return hip_status(e, "render launch");
}

// Host-side table of the scratch array's device address per GPU (see the array's comment at the
// top of this file).
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

hipError_t noalloc_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || !aligned(p, 256)) return hipErrorInvalidSymbol;
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace grafx

using namespace grafx;

extern "C" {

grafx_status grafx_plan_upload(const grafx_schedule_t* h, void* dev_plan, size_t bytes,
                               hipStream_t stream) {
  clear_error();
  if (!h || !dev_plan) return fail(GRAFX_E_ARG, "NULL argument");
  const size_t need = h->layout.total * sizeof(int32_t);
  if (bytes < need) return fail(GRAFX_E_WORKSPACE, "plan buffer too small");
  if (!aligned(dev_plan, 256)) return fail(GRAFX_E_SHAPE, "plan must be 256-byte aligned");
  if (need == 0) return GRAFX_OK;
  return hip_status(hipMemcpyAsync(dev_plan, h->plan.data(), need, hipMemcpyHostToDevice, stream),
                    "plan upload");
}

grafx_status grafx_workspace_bytes(const grafx_schedule_t* h, int64_t T, int32_t with_backward,
                                   size_t* bytes) {
  clear_error();
  if (!h || !bytes) return fail(GRAFX_E_ARG, "NULL argument");
  if (T < 1) return fail(GRAFX_E_SHAPE, "T must be >= 1");
  *bytes = ws_layout(h, T, with_backward != 0).total;
  return GRAFX_OK;
}

grafx_status grafx_render(const grafx_schedule_t* h, const void* dev_plan, int64_t T,
                          const float* S, const float* const* P, float* U, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
  clear_error();
  grafx_status st = check_common(h, dev_plan, T, S, P, U, ws, ws_bytes, false);
  if (st != GRAFX_OK) return st;
  return enqueue_render(h, dev_plan, T, S, P, U, ws, stream);
}

grafx_status grafx_render_noalloc(const grafx_schedule_t* h, const void* dev_plan, int64_t T,
                                  const float* S, const float* const* P, float* U,
                                  hipStream_t stream) {
  clear_error();
  // the same checks as grafx_render with a stand-in workspace of the scratch's size (aligned, not
  // dereferenced), so that a request beyond the scratch fails before any HIP call
  void* const stand_in = reinterpret_cast<void*>(uintptr_t{256});
  grafx_status st = check_common(h, dev_plan, T, S, P, U, stand_in, kNoallocScratchBytes, false);
  if (st == GRAFX_E_WORKSPACE)
    return fail(GRAFX_E_WORKSPACE,
                "grafx_render_noalloc needs " + std::to_string(ws_layout(h, T, false).total) +
                    " bytes of scratch; its static scratch holds " +
                    std::to_string(kNoallocScratchBytes) + " bytes (use grafx_render)");
  if (st != GRAFX_OK) return st;
  void* ws = nullptr;
  st = hip_status(noalloc_scratch(&ws), "scratch address");
  if (st != GRAFX_OK) return st;
  return enqueue_render(h, dev_plan, T, S, P, U, ws, stream);
}

grafx_status grafx_render_backward(const grafx_schedule_t* h, const void* dev_plan, int64_t T,
                                   const float* S, const float* const* P, const float* U,
                                   const float* dY, float* dU, float* dS, float* const* dP,
                                   void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  grafx_status st = check_common(h, dev_plan, T, S, P, U, ws, ws_bytes, true);
  if (st != GRAFX_OK) return st;
  if (!dY || !dU) return fail(GRAFX_E_ARG, "dY or dU is NULL");
  if (!aligned(dY, 16) || !aligned(dU, 16) || (dS && !aligned(dS, 16)))
    return fail(GRAFX_E_SHAPE, "adjoint buffers must be 16-byte aligned");
  const WsLayout L = ws_layout(h, T, true);
  GraphView g = make_view(h, dev_plan, T, S, U);
  g.dY = dY;
  g.dU = dU;
  auto par = [&](int t) -> const float* { return P ? P[t] : nullptr; };
  auto dpar = [&](int t) -> float* { return dP ? dP[t] : nullptr; };
  hipError_t e = reset_comp(h, ws, L, true, T, stream);
  if (e == hipSuccess) e = reset_ar(h, ws, L, true, T, stream);
  for (int n = h->N - 1; n >= 1 && e == hipSuccess; --n)
    e = enqueue_bwd_step(h, g, P, dU, ws, L, n, stream);
  if (e == hipSuccess && dS && h->K > 0)  // adjoint of the input step: sum over output edges
    e = launch_pointwise_bwd(GRAFX_IN, g, dS, nullptr, 0, h->K, nullptr, stream);
  const int tiles = pointwise_tiles(T, h->pw_unroll), chunks = comp_chunks(T);
  ReduceJobs jobs;
  if (dpar(GRAFX_GAIN_PAN))
    jobs.add(at<double>(ws, L.part_gp), h->type_count[GRAFX_GAIN_PAN], tiles, 2,
             dpar(GRAFX_GAIN_PAN));
  if (dpar(GRAFX_IMAGER))
    jobs.add(at<double>(ws, L.part_im), h->type_count[GRAFX_IMAGER], tiles, 1, dpar(GRAFX_IMAGER));
  if (dpar(GRAFX_TANH))
    jobs.add(at<double>(ws, L.part_tanh), h->type_count[GRAFX_TANH], tiles, 1, dpar(GRAFX_TANH));
  for (int t : {GRAFX_COMPRESSOR, GRAFX_NOISEGATE})
    if (dpar(t))
      jobs.add(at<double>(ws, L.comp_part) + (size_t)dyn_row(h, t) * chunks * 4, h->type_count[t],
               chunks, 4, dpar(t));
  if (dpar(GRAFX_COMPRESSOR_AR))
    jobs.add(at<double>(ws, L.ar_part), h->type_count[GRAFX_COMPRESSOR_AR], chunks, kArParams,
             dpar(GRAFX_COMPRESSOR_AR));
  if (e == hipSuccess) e = launch_reduce_partials(jobs, stream);
  if (e == hipSuccess && dpar(GRAFX_EQ))
    e = launch_eq_grad(par(GRAFX_EQ), at<float>(ws, L.eq_C), eq_tiles(T),
                       at<float>(ws, L.eq_spec), h->type_count[GRAFX_EQ],
                       at<double>(ws, L.eq_s), dpar(GRAFX_EQ), stream);
  for (int f = 0; f < 2; ++f) {
    const int t = kDelayType[f], M = kDelaySlots[f], n_del = h->type_count[t];
    if (e != hipSuccess || !dpar(t)) continue;
    e = launch_delay_grad(M, par(t), at<float>(ws, L.delay_part[f]), n_del,
                          delay_groups(T, h->tap_tiles), dpar(t), stream);
    if (e == hipSuccess && h->delay_surrogate)
      // R[n] = sum_t ybar[t - 19] u[t - n] has no term for n >= the node's length + 19
      e = launch_xcorr(n_del, rv_blocks(T + kDelaySurShift), delay_sur_parts(M), delay_sur_len(M),
                       at<int32_t>(ws, L.dl_len[f]), kDelaySurShift,
                       at<float4>(ws, L.dl_Y0[f]), at<float4>(ws, L.dl_X[f]),
                       at<float4>(ws, L.dl_G[f]), at<float>(ws, L.dl_R[f]), stream);
    if (e == hipSuccess && h->delay_surrogate)
      e = launch_delay_phasor_grad(M, par(t), at<float>(ws, L.delay_taps[f]),
                                   at<float>(ws, L.dl_R[f]), n_del, dpar(t), stream);
  }
  if (e == hipSuccess && dpar(GRAFX_REVERB))
    e = launch_rv_grad(h->type_count[GRAFX_REVERB], T, h->rv_len, par(GRAFX_REVERB),
                       at<double2>(ws, L.rv_Un), at<float4>(ws, L.rv_Z), at<float4>(ws, L.rv_Y0),
                       at<int32_t>(ws, L.rv_len), at<float4>(ws, L.rv_G), at<float>(ws, L.rv_hbar), at<double>(ws, L.rv_part),
                       dpar(GRAFX_REVERB), stream);
  return hip_status(e, "render_backward launch");
}

grafx_status grafx_render_step(const grafx_schedule_t* h, const void* dev_plan, int64_t T,
                               const float* S, const float* const* P, float* U, void* ws,
                               size_t ws_bytes, int32_t step, hipStream_t stream) {
  clear_error();
  grafx_status st = check_common(h, dev_plan, T, S, P, U, ws, ws_bytes, false);
  if (st != GRAFX_OK) return st;
  if (step < 1 || step > h->N) return fail(GRAFX_E_ARG, "step out of range");
  const WsLayout L = ws_layout(h, T, false);
  const GraphView g = make_view(h, dev_plan, T, S, U);
  hipError_t e = hipSuccess;
  const bool ar = h->step_type[step] == GRAFX_COMPRESSOR_AR;
  if (is_dynamics(h->step_type[step]) || ar) e = reset_comp(h, ws, L, false, T, stream);
  if (e == hipSuccess && ar) e = reset_ar(h, ws, L, false, T, stream);
  if (e == hipSuccess) e = enqueue_fwd_step(h, g, P, U, ws, L, step, stream);
  return hip_status(e, "render_step launch");
}

grafx_status grafx_render_backward_step(const grafx_schedule_t* h, const void* dev_plan,
                                        int64_t T, const float* S, const float* const* P,
                                        const float* U, const float* dY, float* dU, void* ws,
                                        size_t ws_bytes, int32_t step, hipStream_t stream) {
  clear_error();
  grafx_status st = check_common(h, dev_plan, T, S, P, U, ws, ws_bytes, true);
  if (st != GRAFX_OK) return st;
  if (!dY || !dU) return fail(GRAFX_E_ARG, "dY or dU is NULL");
  if (step < 1 || step >= h->N) return fail(GRAFX_E_ARG, "step out of range");
  const WsLayout L = ws_layout(h, T, true);
  GraphView g = make_view(h, dev_plan, T, S, U);
  g.dY = dY;
  g.dU = dU;
  hipError_t e = hipSuccess;
  if (is_dynamics(h->step_type[step])) e = reset_comp(h, ws, L, true, T, stream);
  if (e == hipSuccess && h->step_type[step] == GRAFX_COMPRESSOR_AR)
    e = reset_ar(h, ws, L, true, T, stream);
  if (e == hipSuccess) e = enqueue_bwd_step(h, g, P, dU, ws, L, step, stream);
  return hip_status(e, "render_backward_step launch");
}

grafx_status grafx_schedule_set_tuning(grafx_schedule_t* h, int32_t knob, int32_t value) {
  clear_error();
  if (!h) return fail(GRAFX_E_ARG, "schedule is NULL");
  switch (knob) {
    case GRAFX_TUNE_POINTWISE_UNROLL:
      if (value != 1 && value != 2 && value != 4)
        return fail(GRAFX_E_ARG, "pointwise unroll must be 1, 2 or 4");
      h->pw_unroll = value;
      return GRAFX_OK;
    case GRAFX_TUNE_AR_MAX_PASSES:
      if (value < 1 || value > kArPasses)
        return fail(GRAFX_E_ARG, "attack/release passes must be in 1.." + std::to_string(kArPasses));
      h->ar_max_pass = value;
      return GRAFX_OK;
    case GRAFX_TUNE_WAIT_POLLS:
      if (value < 0 || value > (1 << 30)) return fail(GRAFX_E_ARG, "wait polls must be in 0..2^30");
      h->wait_polls = value;
      return GRAFX_OK;
    case GRAFX_TUNE_EQ_ORDER:
      if (value != 0 && value != 1) return fail(GRAFX_E_ARG, "EQ block order must be 0 or 1");
      h->eq_order = value;
      return GRAFX_OK;
    case GRAFX_TUNE_DYN_ORDER:
      if (value < 0 || value > 2)
        return fail(GRAFX_E_ARG, "dynamics block order must be 0, 1 or 2");
      h->dyn_order = value;
      return GRAFX_OK;
    case GRAFX_TUNE_TAP_TILES:
      if (value != 4 && value != 8 && value != 16)
        return fail(GRAFX_E_ARG, "delay tap-gradient tiles must be 4, 8 or 16");
      h->tap_tiles = value;
      return GRAFX_OK;
    default:
      return fail(GRAFX_E_ARG, "unknown tuning knob");
  }
}

grafx_status grafx_schedule_set_reverb_noise(grafx_schedule_t* h, const float* noise,
                                            int64_t length) {
  clear_error();
  if (!h) return fail(GRAFX_E_ARG, "schedule is NULL");
  if (!noise) {
    if (length != 0) return fail(GRAFX_E_ARG, "a NULL noise needs length 0");
    h->rv_noise = nullptr;
    h->rv_len = 0;
    return GRAFX_OK;
  }
  if (length < 1 || length > kRvMaxLen)
    return fail(GRAFX_E_SHAPE, "reverb noise length must be in 1.." + std::to_string(kRvMaxLen));
  if (!aligned(noise, 4)) return fail(GRAFX_E_SHAPE, "reverb noise must be 4-byte aligned");
  h->rv_noise = noise;
  h->rv_len = length;
  return GRAFX_OK;
}

grafx_status grafx_delay_phasor_regularise(int32_t delay_type, int32_t n, const float* P,
                                           float* dP, float weight, hipStream_t stream) {
  clear_error();
  if (delay_type != GRAFX_DELAY && delay_type != GRAFX_DELAY_LONG)
    return fail(GRAFX_E_TYPE, "delay_type must be GRAFX_DELAY or GRAFX_DELAY_LONG");
  if (n < 0) return fail(GRAFX_E_SHAPE, "n must be >= 0");
  if (n > 0 && (!P || !dP)) return fail(GRAFX_E_ARG, "P or dP is NULL");
  if (!(weight >= 0.0f) || weight > 3.0e38f)
    return fail(GRAFX_E_ARG, "weight must be finite and >= 0");
  if ((P && !aligned(P, 4)) || (dP && !aligned(dP, 4)))
    return fail(GRAFX_E_SHAPE, "P and dP must be 4-byte aligned");
  return hip_status(launch_delay_phasor_regularise(kDelaySlots[delay_family(delay_type)], n, P,
                                                   dP, weight, stream),
                    "delay_phasor_regularise launch");
}

grafx_status grafx_schedule_set_delay_surrogate(grafx_schedule_t* h, int32_t enable) {
  clear_error();
  if (!h) return fail(GRAFX_E_ARG, "schedule is NULL");
  if (enable != 0 && enable != 1) return fail(GRAFX_E_ARG, "enable must be 0 or 1");
  h->delay_surrogate = enable;
  return GRAFX_OK;
}

grafx_status grafx_schedule_get_tuning(const grafx_schedule_t* h, int32_t knob, int32_t* value) {
  clear_error();
  if (!h || !value) return fail(GRAFX_E_ARG, "NULL argument");
  switch (knob) {
    case GRAFX_TUNE_POINTWISE_UNROLL: *value = h->pw_unroll; return GRAFX_OK;
    case GRAFX_TUNE_AR_MAX_PASSES: *value = h->ar_max_pass; return GRAFX_OK;
    case GRAFX_TUNE_WAIT_POLLS: *value = h->wait_polls; return GRAFX_OK;
    case GRAFX_TUNE_EQ_ORDER: *value = h->eq_order; return GRAFX_OK;
    case GRAFX_TUNE_DYN_ORDER: *value = h->dyn_order; return GRAFX_OK;
    case GRAFX_TUNE_TAP_TILES: *value = h->tap_tiles; return GRAFX_OK;
    default: return fail(GRAFX_E_ARG, "unknown tuning knob");
  }
}

grafx_status grafx_workspace_error(const grafx_schedule_t* h, int64_t T, const void* ws,
                                   size_t ws_bytes, uint32_t* word, hipStream_t stream) {
  clear_error();
  if (!h || !ws || !word) return fail(GRAFX_E_ARG, "NULL argument");
  if (T < 1 || T >= ((int64_t)1 << 29)) return fail(GRAFX_E_SHAPE, "T must be in [1, 2^29)");
  if (!aligned(ws, 256)) return fail(GRAFX_E_SHAPE, "workspace must be 256-byte aligned");
  const WsLayout L = ws_layout(h, T, false);
  if (ws_bytes < L.fwd_end)
    return fail(GRAFX_E_WORKSPACE, "workspace too small: need " + std::to_string(L.fwd_end) +
                                       " bytes, got " + std::to_string(ws_bytes));
  static const uint32_t kZero = 0;
  const void* src = has_dynamics(h) ? static_cast<const void*>(
                                          error_word(const_cast<void*>(ws), L))
                                    : static_cast<const void*>(&kZero);
  return hip_status(hipMemcpyAsync(word, src, sizeof(uint32_t), hipMemcpyDefault, stream),
                    "error word copy");
}

grafx_status grafx_mrstft_workspace_bytes(int32_t rows, int64_t T, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(GRAFX_E_ARG, "NULL argument");
  if (rows < 1 || T < 1) return fail(GRAFX_E_SHAPE, "rows and T must be >= 1");
  *bytes = mrstft_ws_bytes(rows, T);
  return GRAFX_OK;
}

static grafx_status check_mrstft(int32_t rows, int64_t T, const float* Y, const float* tgt,
                                 void* ws, size_t ws_bytes) {
  if (rows < 1 || T < 1) return fail(GRAFX_E_SHAPE, "rows and T must be >= 1");
  if (!Y || !tgt || !ws) return fail(GRAFX_E_ARG, "NULL argument");
  if (ws_bytes < mrstft_ws_bytes(rows, T)) return fail(GRAFX_E_WORKSPACE, "workspace too small");
  if (!aligned(ws, 256)) return fail(GRAFX_E_SHAPE, "workspace must be 256-byte aligned");
  return GRAFX_OK;
}

grafx_status grafx_mrstft_loss(int32_t rows, int64_t T, const float* Y, const float* target,
                               float* loss, void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  grafx_status st = check_mrstft(rows, T, Y, target, ws, ws_bytes);
  if (st != GRAFX_OK) return st;
  if (!loss) return fail(GRAFX_E_ARG, "loss is NULL");
  return hip_status(launch_mrstft_loss(rows, T, Y, target, loss, ws, stream), "mrstft launch");
}

grafx_status grafx_mrstft_backward(int32_t rows, int64_t T, const float* Y, const float* target,
                                   const float* dloss, float* dY, void* ws, size_t ws_bytes,
                                   hipStream_t stream) {
  clear_error();
  grafx_status st = check_mrstft(rows, T, Y, target, ws, ws_bytes);
  if (st != GRAFX_OK) return st;
  if (!dloss || !dY) return fail(GRAFX_E_ARG, "dloss or dY is NULL");
  return hip_status(launch_mrstft_bwd(rows, T, Y, target, dloss, dY, ws, stream),
                    "mrstft_backward launch");
}

}  // extern "C"
