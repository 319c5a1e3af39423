// Host-side launchers of the device kernels (one translation unit per processor family).
// Every launcher only enqueues work on the given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace grafx {

struct GraphView;

// ---- pointwise family: mix / out / gain_pan / imager / tanh (k_pointwise.hip) --------------
// blocks per node along time (partials per node) when every thread covers `unroll` float4 groups
int pointwise_tiles(int64_t T, int unroll = 1);
hipError_t launch_pointwise_fwd(int type, const GraphView& g, float* U, const float* P,
                                int node_begin, int n_nodes, hipStream_t s);
// dst: dU (or dS for the input step); part: double [slots][tiles][NP] (NP = 2, 1, 1, 0)
hipError_t launch_pointwise_bwd(int type, const GraphView& g, float* dst, const float* P,
                                int node_begin, int n_nodes, double* part, hipStream_t s);
// Fixed-order sums of per-tile parameter-gradient partials, several parameter types in one
// launch: job q reduces part[q] [slots][tiles][np] (double) into dP[q] [slots][np] (float).
struct ReduceJobs {
  static constexpr int kMax = 8;
  const double* part[kMax];
  float* dP[kMax];
  int slots[kMax], tiles[kMax], np[kMax];
  int n = 0;
  void add(const double* p, int n_slots, int n_tiles, int n_par, float* out) {
    if (n_slots <= 0) return;
    part[n] = p;
    dP[n] = out;
    slots[n] = n_slots;
    tiles[n] = n_tiles;
    np[n] = n_par;
    ++n;
  }
};
hipError_t launch_reduce_partials(const ReduceJobs& jobs, hipStream_t s);

// ---- EQ (k_eq.hip) ---------------------------------------------------------------------------
constexpr int kEqFFT = 4096;  // overlap-save FFT size
constexpr int kEqHop = 2048;  // outputs per tile
int eq_tiles(int64_t T);
constexpr int kEqFoldStride = 2112;  // N/2 + 1 = 2049 folded bins, padded to 256 bytes
// h: double [n_eq][1024] (windowed FIR, taps n = 0..1023; even), H: float [n_eq][4096]
hipError_t launch_eq_design(const float* P, int n_eq, double* h, float* H, hipStream_t s);
hipError_t launch_eq_fwd(const GraphView& g, float* U, const float* H, int node_begin,
                         int n_nodes, hipStream_t s);
// Adjoint of one step. Fpart: float [n_eq][tiles][kEqFoldStride]: the regions (by parameter
// slot) of the step's nodes are written, one folded cross-spectrum per tile.
hipError_t launch_eq_bwd(const GraphView& g, float* dU, const float* H, int node_begin,
                         int n_nodes, float* Fpart, hipStream_t s);
// After the last adjoint step: the tiles of Fpart summed per slot into F (float
// [n_eq][kEqFoldStride]), then the FIR and parameter gradients; sbuf: double [n_eq][1024]
// scratch; dP: float [n_eq][1024]
hipError_t launch_eq_grad(const float* P, const float* Fpart, int tiles, float* F, int n_eq,
                          double* sbuf, float* dP, hipStream_t s);

// ---- compressor (k_comp.hip) ---------------------------------------------------------------
constexpr int kCompChunk = 3072;  // 256 threads x 12 samples
int comp_chunks(int64_t T);
// agg, ragg: uint64 [n_comp][chunks] published chunk totals (reset to "not ready" before each
// pass); carry: double [n_comp][chunks] envelope entering each chunk (forward, kept for the
// adjoint); part: double [n_comp][chunks][4]; ticket: one counter per compressor node (reset to 0),
// kCompTicketStride words apart so that no two counters share a cache line (atomics on one line
// serialise); err: error word (bit 0: a wait ran out, bit 1: tickets were not reset)
constexpr int kCompTicketStride = 64;
hipError_t launch_comp_reset(uint64_t* tot, int64_t n, unsigned* tickets, int n_tickets,
                             hipStream_t s);
// Compressors and noisegates share one workspace family ("dynamics"): rows [0, n_comp) belong to
// the compressors, [n_comp, n_comp + n_gate) to the noisegates; ws_off is the family row of the
// launch's type (0 or n_comp) and `gate` selects the noisegate curve.
hipError_t launch_comp_fwd(const GraphView& g, float* U, const float* P, int node_begin,
                           int n_nodes, int ws_off, bool gate, uint64_t* agg, double* carry,
                           unsigned* ticket, unsigned* err, hipStream_t s);
hipError_t launch_comp_bwd(const GraphView& g, float* dU, const float* P, int node_begin,
                           int n_nodes, int ws_off, bool gate, const double* carry,
                           uint64_t* ragg, double* part, unsigned* ticket, unsigned* err,
                           hipStream_t s);

// ---- compressor with attack/release ballistics (k_comp_ar.hip) -----------------------------
constexpr int kArParams = 5;   // alpha_a, alpha_r, T, W, R
constexpr int kArPasses = 16;  // branch-pattern passes before a chunk falls back to the serial loop
// pslot: uint64 [n_ar][kArPasses][chunks][3] and fin: uint64 [n_ar][chunks][2], both reset to
// "not ready"; carry: double [n_ar][chunks] and pats: uint16 [n_ar][chunks][kBlock] are written
// for the adjoint; ragg: uint64 [n_ar][chunks][2] (reset); part: double [n_ar][chunks][5];
// ticket: kCompTicketStride words per node (reset to 0); err as for the compressor.
hipError_t launch_comp_ar_fwd(const GraphView& g, float* U, const float* P, int node_begin,
                              int n_nodes, int max_pass, uint64_t* pslot, uint64_t* fin,
                              double* carry, uint16_t* pats, unsigned* ticket, unsigned* err,
                              hipStream_t s);
hipError_t launch_comp_ar_bwd(const GraphView& g, float* dU, const float* P, int node_begin,
                              int n_nodes, const double* carry, const uint16_t* pats,
                              uint64_t* ragg, double* part, unsigned* ticket, unsigned* err,
                              hipStream_t s);

// ---- delay (k_delay.hip) -------------------------------------------------------------------
// M 100 ms slots per channel: M = 5 (node type delay, 500 ms) or M = 20 (delay_long, 2 s).
constexpr int kDelayTaps = 5, kDelayTapsLong = 20, kDelayFir = 39, kDelaySlot = 4410;
constexpr int delay_coef(int M) { return 2 * M * kDelayFir; }  // filter taps per node
constexpr int delay_row(int M) { return 2 * M * 22; }          // parameters per node
int delay_tiles(int64_t T);
constexpr int kTapTilesMin = 4;  // smallest tap-gradient group (sizes the partials)
int delay_groups(int64_t T, int tap_tiles);  // tile groups per node in the tap-gradient pass
// taps: float [n][delay_coef(M)]; offs: int32 [n][2 M]
hipError_t launch_delay_design(int M, const float* P, int n, float* taps, int32_t* offs,
                               hipStream_t s);
hipError_t launch_delay_fwd(int M, const GraphView& g, float* U, const float* taps,
                            const int32_t* offs, int node_begin, int n_nodes, hipStream_t s);
// part: float [n][groups][delay_coef(M)]
hipError_t launch_delay_bwd(int M, const GraphView& g, float* dU, const float* taps,
                            const int32_t* offs, int node_begin, int n_nodes, float* part,
                            hipStream_t s);
hipError_t launch_delay_grad(int M, const float* P, const float* part, int n, int groups,
                             float* dP, hipStream_t s);
// Delay-time surrogate: lags -19 .. M x 4410 + 19 of the input/adjoint cross-correlation (the
// output adjoint delayed by kDelaySurShift, so that the lags start at 0), rounded up to whole
// 2048-lag partitions (M = 5: 11 partitions; M = 20: 44)
constexpr int kDelaySurShift = (kDelayFir - 1) / 2;  // 19
constexpr int delay_sur_parts(int M) { return (M * kDelaySlot + kDelayFir - 1 + 2047) / 2048; }
constexpr int64_t delay_sur_len(int M) { return (int64_t)delay_sur_parts(M) * 2048; }
// R: float [n][2][delay_sur_len(M)] correlation (launch_xcorr); writes the phasor entries of dP
// (after launch_delay_grad, which sets them to 0)
hipError_t launch_delay_phasor_grad(int M, const float* P, const float* taps, const float* R,
                                    int n, float* dP, hipStream_t s);
// dP phasor entries: unit-length per phasor, plus the gradient of weight * (|z| - 1)^2
hipError_t launch_delay_phasor_regularise(int M, int n, const float* P, float* dP, float weight,
                                          hipStream_t s);

// ---- reverb (k_reverb.hip) ------------------------------------------------------------------
constexpr int kRvFft = 384, kRvHop = 192;  // STFT of the noise and of the masks
constexpr int kRvBins = 192;               // parameterised one-sided bins (bin 192 takes 191's)
constexpr int kRvParams = 4 * kRvBins;     // [mid, side][H0, HD][bins] = 768
constexpr int kRvBlock = 2048;             // FIR partition length and output block length
constexpr int kRvHalf = 2049;              // one-sided bins of the 4096-point block transforms
constexpr int kRvStride = 2064;            // float4 entries per stored spectrum (256-byte rows)
int rv_frames(int64_t L);  // STFT frames of an L-sample noise
int rv_parts(int64_t L);   // FIR partitions of an L-tap response
int rv_blocks(int64_t T);  // output blocks of a T-sample row
int rv_grad_blocks(int64_t L);  // blocks of the mask-gradient pass (frames in groups of 8)
// noise: float [2][L] (mid, side); Un: double2 [2][frames][193] (noise STFT); h: float
// [n][2][L] (left, right FIR); Hs: float4 [n][parts][kRvStride] (per-channel one-sided partition
// spectra (left re, left im, right re, right im), scaled by 1 / 4096)
hipError_t launch_rv_design(const float* P, int n, const float* noise, int64_t L, double2* Un,
                            float* h, float4* Hs, hipStream_t s);
// Z: float4 [n][blocks][kRvStride] per-channel one-sided spectra of the input windows (kept for
// the adjoint); C: float4 [n][rv_conv_tiles(L)][blocks][kRvStride] partial product spectra
// (scratch, shared by the forward and the adjoint)
int rv_conv_tiles(int64_t L);
hipError_t launch_rv_fwd(const GraphView& g, float* U, int node_begin, int n_nodes, int64_t L,
                         const float4* Hs, float4* Z, float4* C, hipStream_t s);
// Y0: float4 [n][blocks][kRvStride] spectra of the output-adjoint blocks (kept for the FIR
// gradient)
hipError_t launch_rv_bwd(const GraphView& g, float* dU, int node_begin, int n_nodes, int64_t L,
                         const float4* Hs, float4* Y0, float4* C, int32_t* slot_len,
                         hipStream_t s);
// Partitioned cross-correlation R_c[n] = sum_t ybar_c[t + s_a] u_c[t + s_i - n], n in [0, len),
// of a node's output adjoint and its input sum (the reverb's FIR gradient; the delay's surrogate
// gradient), over nb blocks of 2048 (nb x 2048 must cover every t with a non-zero term). Spectra
// per node parameter slot: input windows (adj false, shift s_i: [2048 b - 2048 + s_i,
// 2048 b + 2048 + s_i)) or single output-adjoint blocks (adj true, shift s_a:
// [2048 b + s_a, 2048 b + 2048 + s_a)), float4 [slots][nb][kRvStride], and, if slot_len is not
// null, each node's length at its slot; then, for n slots, Gs: float4 [n][parts][kRvStride]
// cross-spectra and R: float [n][2][len] (parts = ceil(len / 2048)); lags from
// valid_len[slot] + valid_shift on (where no term of the sum exists) are stored as exact zeros.
// Input samples before 0 must not reach a term (s_i <= 0): the input windows start at b = 0.
hipError_t launch_xcorr_spectra(const GraphView& g, int node_begin, int n_nodes, bool adj,
                                int shift, int nb, float4* out, int32_t* slot_len, hipStream_t s);
hipError_t launch_xcorr(int n, int nb, int parts, int64_t len, const int32_t* valid_len,
                        int valid_shift, const float4* Y0, const float4* X, float4* Gs, float* R,
                        hipStream_t s);
// After the last adjoint step, every reverb slot: Gs: float4 [n][parts][kRvStride] partition
// cross-spectra; hbar: float [n][2][L]; part: double [n][grad blocks][2][193][2]; dP: float
// [n][768]
hipError_t launch_rv_grad(int n, int64_t T, int64_t L, const float* P, const double2* Un,
                          const float4* Z, const float4* Y0, const int32_t* slot_len, float4* Gs,
                          float* hbar, double* part, float* dP, hipStream_t s);

// ---- MRSTFT loss (k_mrstft.hip) -------------------------------------------------------------
size_t mrstft_ws_bytes(int rows, int64_t T);
hipError_t launch_mrstft_loss(int rows, int64_t T, const float* Y, const float* tgt, float* loss,
                              void* ws, hipStream_t s);
// log-mel features [n_sig][128][F] of stereo signals [n_sig][2][T] (frames of 1024 at hop 256)
int logmel_frames(int64_t T);
hipError_t launch_logmel(int n_sig, int64_t T, const float* sig, float* feats, hipStream_t s);
hipError_t launch_mrstft_bwd(int rows, int64_t T, const float* Y, const float* tgt,
                             const float* dloss, float* dY, void* ws, hipStream_t s);

}  // namespace grafx
