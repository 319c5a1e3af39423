// Internal definitions shared by the host scheduler, the render drivers and the kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "grafx.h"

namespace grafx {

constexpr int kNumTypes = GRAFX_NUM_TYPES;
constexpr int64_t kRvMaxLen = GRAFX_REVERB_MAX_LEN;
constexpr int kParamCount[kNumTypes] = {0, 0, 0, 2, 1024, 4, 1, 220, 1, 4, 5, 768, 880};

// Thread-local error message, set by every failing entry point.
grafx_status fail(grafx_status code, const std::string& msg);
void clear_error();

// Round up to a multiple of `a` (a power of two).
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) & ~(a - 1); }

// Device plan layout: int32 sections, each starting on a 64-element (256-byte) boundary.
struct PlanLayout {
  size_t in_ptr, in_src, out_ptr, out_dst, param_row;  // element offsets
  size_t len;                                            // per-node lengths (if any)
  size_t total;                                          // elements
};

}  // namespace grafx

// The schedule handle (host memory only). Its graph and plan are immutable after creation; only
// the settings (grafx_schedule_set_tuning) change.
struct grafx_schedule_t {
  int32_t V = 0, E = 0, N = 0, K = 0, n_out = 0;
  int32_t type_count[grafx::kNumTypes] = {0};
  std::vector<int32_t> node_type;  // original order
  std::vector<int32_t> step_type;  // [N+1]
  std::vector<int32_t> step_ptr;   // [N+2]
  std::vector<int32_t> perm;       // [V]
  std::vector<int32_t> in_ptr;     // [V+1]
  std::vector<int32_t> in_src;     // [E]
  std::vector<int32_t> out_ptr;    // [V+1]
  std::vector<int32_t> out_dst;    // [E]
  std::vector<int32_t> param_row;  // [V]
  std::vector<int32_t> node_len;   // [V] per-node signal length (sigma order); empty = all T
  int32_t max_len = 0;             // largest node length (0 when uniform)
  bool len4 = true;                // every node length is a multiple of 4
  int32_t pw_unroll = 1;           // tuning: pointwise 1024-sample parts per block
  int32_t ar_max_pass = 16;        // attack/release forward: branch-pattern passes (1..16)
  int32_t wait_polls = 1 << 24;    // dynamics kernels: polls of a chunk wait before giving up
  int32_t eq_order = 0;            // tuning: EQ block order (0 XCD-contiguous, 1 hardware order)
  int32_t dyn_order = 2;           // tuning: dynamics block order (0 node-major, 1 interleaved,
                                   // 2 interleaved only for launches of many blocks)
  int32_t tap_tiles = 16;          // tuning: delay tiles per tap-gradient block (4, 8 or 16)
  const float* rv_noise = nullptr; // reverb noise realisation (device, [2][rv_len]; borrowed)
  int64_t rv_len = 0;              // its length: the reverb FIR length
  int32_t delay_surrogate = 0;     // delay phasors: 0 no gradient, 1 straight-through surrogate
  grafx::PlanLayout layout{};
  std::vector<int32_t> plan;       // packed host image of the device plan
};
