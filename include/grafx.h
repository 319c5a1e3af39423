/*
 * grafx.h -- C ABI of libgrafx: batched forward render and adjoint of an audio processing graph
 * on one AMD MI355X (gfx950).
 *
 * The data contract follows the paper's tensor representation of a graph (GRAFX, Lee et al.,
 * DAFx-24, arXiv 2408.03204, Sec. 2 "Graph representations"): a node type vector T_V, an edge
 * index E (2 x |E|), an optional edge type tensor T_E, one parameter matrix P[t] per node type
 * (|V_t| rows, N_t columns) and a source tensor S (K x C x L), all in one shared node order: the
 * k-th source feeds the k-th input node, the l-th row of P[t] belongs to the l-th type-t node.
 * The render follows Algorithm 1 of the paper: schedule, reorder, build read/write indices
 * (host, grafx_schedule), then one batched processor call per schedule step on the GPU
 * (grafx_render). grafx_render_backward is the adjoint of grafx_render.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns a grafx_status. On an error, grafx_last_error() gives a message for the
 *   calling thread, and the call has had no side effect: all arguments are checked before any
 *   device work is enqueued.
 * - Ownership: the caller owns all device memory (plan, signal buffers, workspaces, gradients);
 *   the library never allocates or frees device memory and never synchronises a stream (its one
 *   device array, the scratch of grafx_render_noalloc, is part of its code object). A
 *   schedule handle owns host memory only; its graph and plan are immutable after creation, and
 *   it may be shared by threads and streams. Its settings (tuning knobs, the reverb noise, the
 *   delay-time gradient) are changed only by the grafx_schedule_set_* calls.
 * - Device work is enqueued on the caller's stream and runs asynchronously. Two calls that share
 *   a workspace must be ordered on one stream (or otherwise synchronised) by the caller.
 * - Signals are float32, stereo (C = 2), time-contiguous: a node's row is [2][T] (channel-major,
 *   time fastest); node rows are contiguous.
 * - Any T >= 1 is accepted.
 *
 * Node types (codes) and parameter rows (N_t floats per node):
 *   0 in         --   emits its source row of S
 *   1 out        --   sum of inputs; the graph outputs Y
 *   2 mix        --   sum of inputs
 *   3 gain_pan   2    y_c = exp(p_c) u_c                                  (paper Eq. 2)
 *   4 eq         1024 zero-phase 2047-tap FIR from 1024 log-magnitudes    (Eqs. 4-5)
 *   5 compressor 4    (alpha, T, W, R): one-pole energy envelope, quadratic knee (Eqs. 8-12);
 *                     alpha in [0, 1) (the envelope of a negative alpha can go negative and
 *                     its log is NaN, as in Eq. 11); W <= 0 is a hard knee; R > 0
 *   6 imager     1    mid/side width                                     (Eq. 3)
 *   7 delay      220  [channel 2][slot 5][re z, im z, 20 log-magnitudes]  (Eq. 14, <= 500 ms)
 *   8 tanh       1    y = tanh(exp(p) u)                                  (not in the paper)
 *   9 noisegate  4    (alpha, T, W, R): the compressor's envelope with a downward-expander
 *                     curve, ratio R >= 1 below T - W, quadratic knee   (Sec. 3 "Noisegate")
 *  10 compressor_ar 5 (alpha_a, alpha_r, T, W, R): the compressor with distinct attack and
 *                     release coefficients, alpha_a while x[t] > g[t-1]  (Eq. 8 unrestricted)
 *  11 reverb     768  [mid, side][H0, HD][192 bins]: filtered-noise mid/side reverb (Eqs. 6-7),
 *                     a causal stereo FIR made from the noise of grafx_schedule_set_reverb_noise
 *  12 delay_long 880  [channel 2][slot 20][re z, im z, 20 log-magnitudes]: the multitap delay
 *                     with the paper's 20 slots of 100 ms (2 s)                (Eq. 14)
 * The node input is the sum over incoming edges of the source node outputs (Eq. 1b), parallel
 * edges counted once each, summed in original edge order.
 */
#ifndef GRAFX_H_
#define GRAFX_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum grafx_status {
  GRAFX_OK = 0,
  GRAFX_E_ARG = 1,       /* null pointer, negative count, bad method or beam width         */
  GRAFX_E_GRAPH = 2,     /* edge to a missing node, edge into `in`, out of `out`, no `out` */
  GRAFX_E_CYCLE = 3,     /* the graph has a cycle                                          */
  GRAFX_E_TYPE = 4,      /* unknown node type, or a non-zero edge type (SISO only)         */
  GRAFX_E_SHAPE = 5,     /* T < 1, size mismatch, misaligned buffer, missing parameters    */
  GRAFX_E_LIMIT = 6,     /* optimal schedule search exceeded its state limit               */
  GRAFX_E_WORKSPACE = 7, /* workspace or plan buffer too small                             */
  GRAFX_E_HIP = 8        /* a HIP runtime call or kernel launch failed                     */
} grafx_status;

enum {
  GRAFX_IN = 0, GRAFX_OUT = 1, GRAFX_MIX = 2, GRAFX_GAIN_PAN = 3, GRAFX_EQ = 4,
  GRAFX_COMPRESSOR = 5, GRAFX_IMAGER = 6, GRAFX_DELAY = 7, GRAFX_TANH = 8, GRAFX_NOISEGATE = 9,
  GRAFX_COMPRESSOR_AR = 10, GRAFX_REVERB = 11, GRAFX_DELAY_LONG = 12, GRAFX_NUM_TYPES = 13
};

/* Schedule search methods (paper Sec. 2 "Type scheduling"; Sec. 4 "Speed benchmark"). */
typedef enum grafx_sched_method {
  GRAFX_SCHED_ONE_BY_ONE = 0, /* one node per step: the ready node with the smallest id        */
  GRAFX_SCHED_GREEDY = 1,     /* the type with the most ready nodes, ties to the smallest code */
  GRAFX_SCHED_BEAM = 2,       /* beam search over type strings (32 in the paper's benchmark)   */
  GRAFX_SCHED_OPTIMAL = 3     /* exhaustive breadth-first search over computed-node sets       */
} grafx_sched_method;

typedef struct grafx_schedule_t grafx_schedule_t; /* opaque; host memory only */

typedef struct grafx_schedule_sizes {
  int32_t num_nodes;   /* |V|                                                  */
  int32_t num_edges;   /* |E|                                                  */
  int32_t num_steps;   /* N: steps 0..N; step 0 = inputs, step N = outputs     */
  int32_t num_inputs;  /* K                                                    */
  int32_t num_outputs; /* |V_N|                                                */
  int32_t type_count[GRAFX_NUM_TYPES]; /* nodes per type                       */
  int64_t plan_bytes;  /* device bytes needed by grafx_plan_upload             */
  int64_t max_len;     /* largest per-node length (grafx_schedule_with_lengths); 0 otherwise */
} grafx_schedule_sizes;

/*
 * grafx_schedule -- ScheduleBatchedProcessing, OptimizeNodeOrder, Reorder and GetReadWriteIndex
 * of Algorithm 1 (paper Sec. 2, "Type scheduling" and "Implementation details"), on the host.
 *
 * Splits the nodes into steps V_0..V_N that form a partition, are causal and hold one type each
 * (Sec. 2, "Batched processing"); V_0 holds every input and V_N every output node. For the
 * greedy, beam and optimal methods each step is the maximal set of ready nodes of its type, so a
 * schedule is a type string. Ties: greedy prefers the smallest type code; a beam keeps, per set
 * of computed nodes, the lexicographically smallest string, ranks by (more nodes computed, then
 * smaller string) and keeps `beam_width` states; it ends at the first depth where a state has
 * computed every non-output node, choosing the smallest such string. Optimal is the beam without
 * a width cap. Nodes are then reordered by (step, original id) ("sigma"), and the read/write
 * index lists are built as CSR arrays in that order.
 *
 *   num_nodes, node_type    host int32[num_nodes], codes 0..12 (the node types above)
 *   num_edges, edge_src/dst host int32[num_edges] each (may be NULL when num_edges == 0)
 *   edge_type               host int32[2*num_edges] or NULL; must be all zero (SISO graphs)
 *   method                  grafx_sched_method
 *   beam_width              >= 1, used by GRAFX_SCHED_BEAM only
 *   state_limit             >= 1, used by GRAFX_SCHED_OPTIMAL only: the search fails with
 *                           GRAFX_E_LIMIT when more states than this are live at one depth
 *   out                     receives a new handle; release it with grafx_schedule_free
 * Errors: GRAFX_E_ARG, GRAFX_E_TYPE, GRAFX_E_GRAPH, GRAFX_E_CYCLE, GRAFX_E_LIMIT (checked in
 * that order: types, edge endpoints, edge types, edge directions, outputs, cycles, search).
 */
grafx_status grafx_schedule(int32_t num_nodes, const int32_t* node_type, int32_t num_edges,
                            const int32_t* edge_src, const int32_t* edge_dst,
                            const int32_t* edge_type, int32_t method, int32_t beam_width,
                            int64_t state_limit, grafx_schedule_t** out);

/*
 * grafx_schedule_with_lengths -- grafx_schedule for a graph whose nodes carry signals of
 * different lengths: several graphs of different T merged into one schedule (the graph-level
 * parallelism of paper Sec. 2, "Batched processing": a batch of graphs is one disconnected
 * graph). Node v's signal is defined on [0, node_len[v]) and is zero beyond: an input node's
 * source row holds node_len[v] valid samples, every processor sees its inputs as zero past their
 * lengths, and a processed node's row is computed and written on [0, node_len[v]) only (samples
 * at or beyond the length are not written). The T passed to the render calls is then the row
 * stride of S, U, dY and dU and must be >= every length. On a graph whose nodes all have length
 * T the results equal grafx_schedule's bit for bit. Both ends of every edge must have the same
 * length (each connected graph has one length), so every graph of a merged batch renders exactly
 * as it would alone at its own T.
 *
 *   node_len  host int32[num_nodes] in node order, each in [1, 2^29)
 *   (other arguments and errors as grafx_schedule; GRAFX_E_SHAPE for a length out of range or an
 *   edge between nodes of different lengths)
 */
grafx_status grafx_schedule_with_lengths(int32_t num_nodes, const int32_t* node_type,
                                         int32_t num_edges, const int32_t* edge_src,
                                         const int32_t* edge_dst, const int32_t* edge_type,
                                         const int32_t* node_len, int32_t method,
                                         int32_t beam_width, int64_t state_limit,
                                         grafx_schedule_t** out);

/*
 * grafx_set_schedule_threads -- host threads that the beam and optimal searches of later
 * grafx_schedule / grafx_schedule_with_lengths calls (on any thread) may use. The preprocessing
 * runs on the CPU off the GPU's path, in several threads (paper Sec. 2, "Implementation
 * details"): a search depth with enough work (states x processing nodes >= 65536) is split into
 * contiguous slices of states, one per thread, and the children are merged in the serial order,
 * so every thread count gives the same schedule bit for bit.
 *   n >= 1   use at most n threads per search
 *   n == 0   restore the default: the host's hardware concurrency, at most 16
 *   n < 0    leave the setting unchanged (a query)
 * Returns the setting before the call (0 for the default). Never fails.
 */
int32_t grafx_set_schedule_threads(int32_t n);

/*
 * grafx_schedule_free -- release a handle made by grafx_schedule or grafx_schedule_with_lengths
 * (the host copy of the preprocessing results of Algorithm 1: the type string, the reordering
 * sigma and the read/write indices). NULL is ignored. The caller must not free a handle that a
 * call on another thread still uses, nor before a grafx_plan_upload copy from it has completed.
 */
void grafx_schedule_free(grafx_schedule_t* sched);

/*
 * grafx_schedule_query -- sizes of a schedule (host only): |V|, |E|, the number N of processing
 * steps after the input step (the length of the type string minus one, paper Sec. 2 "Type
 * scheduling": steps V_0..V_N), the input count K (Sec. 2 "Graph representations": the k-th
 * source feeds the k-th input node), the output count |V_N| (the rows of Y, Algorithm 1 Ensure),
 * the nodes per type (the rows each P[t] must have, Algorithm 1 Require), the device bytes of
 * the plan and the largest per-node length.
 * Errors: GRAFX_E_ARG for a NULL argument. Never touches the device.
 */
grafx_status grafx_schedule_query(const grafx_schedule_t* sched, grafx_schedule_sizes* out);

/*
 * grafx_schedule_export -- host copies of the outputs of ScheduleBatchedProcessing,
 * OptimizeNodeOrder and GetReadWriteIndex of Algorithm 1 (paper Sec. 2, "Implementation
 * details"): the type string, the reordering sigma, and the gather (I^G), aggregate (I^A),
 * parameter (I^P) and store (I^S) indices, here in CSR form over sigma positions. Every pointer
 * may be NULL to skip that array; the caller owns the arrays, sized as below from
 * grafx_schedule_query. Errors: GRAFX_E_ARG for a NULL schedule.
 *   step_type int32[N+1]  type of each step (step 0 = in, step N = out)
 *   step_ptr  int32[N+2]  step n holds reordered positions [step_ptr[n], step_ptr[n+1])
 *   perm      int32[V]    perm[i] = original id of the node at reordered position i
 *   in_ptr    int32[V+1], in_src int32[E]: inputs of position i, as reordered positions of the
 *                         sources, in original edge order (the gather/aggregate indices)
 *   out_ptr   int32[V+1], out_dst int32[E]: outputs of position i, as reordered positions
 *   param_row int32[V]    row of position i's node in P[type] (and, for inputs, in S; for
 *                         outputs, in Y)
 */
grafx_status grafx_schedule_export(const grafx_schedule_t* sched, int32_t* step_type,
                                   int32_t* step_ptr, int32_t* perm, int32_t* in_ptr,
                                   int32_t* in_src, int32_t* out_ptr, int32_t* out_dst,
                                   int32_t* param_row);

/*
 * grafx_plan_upload -- copy the read/write indices of GetReadWriteIndex (Algorithm 1; I^G and
 * I^A as the in-CSR, its mirror for the adjoint, I^P as param_row, and per-node lengths if any)
 * to caller-owned device memory `dev_plan` (>= plan_bytes bytes, 256-byte aligned) with an
 * asynchronous host-to-device copy on `stream`; the main loop of Algorithm 1 reads them there.
 * The host arrays belong to the handle, which must outlive the copy.
 * Errors: GRAFX_E_ARG (NULL schedule or plan), GRAFX_E_WORKSPACE (bytes < plan_bytes),
 * GRAFX_E_SHAPE (misaligned plan), GRAFX_E_HIP (the copy could not be enqueued).
 */
grafx_status grafx_plan_upload(const grafx_schedule_t* sched, void* dev_plan, size_t bytes,
                               hipStream_t stream);

/*
 * grafx_workspace_bytes -- device workspace bytes for grafx_render (with_backward = 0) or for a
 * render followed by grafx_render_backward on the same workspace (with_backward = 1), for
 * signals of length (row stride) T. The workspace holds what the Process step of Algorithm 1
 * derives from the parameters P (EQ and delay filter designs, Eqs. 4 and 14), the compressor
 * chunk states of Eq. 8, and, for the adjoint, the per-tile parameter-gradient partials. Its
 * size depends only on the schedule's node counts and on T; the caller allocates it (the
 * library never allocates device memory). Errors: GRAFX_E_ARG (NULL argument), GRAFX_E_SHAPE
 * (T < 1).
 */
grafx_status grafx_workspace_bytes(const grafx_schedule_t* sched, int64_t T,
                                   int32_t with_backward, size_t* bytes);

/*
 * grafx_render -- the batched render loop of Algorithm 1 (paper Sec. 2, "Implementation
 * details"): for each step n = 1..N, gather and sum the inputs of the step's nodes from U,
 * run the step's processor on all of them at once with their parameter rows, store the outputs
 * in U.
 *
 *   dev_plan  device copy of the plan (grafx_plan_upload)
 *   T         signal length (samples per channel), >= 1
 *   S         device float32 [K][2][T], sources in node order of the input nodes
 *   P         host array of GRAFX_NUM_TYPES device pointers; P[t] is float32 [|V_t|][N_t], rows
 *             in node order (the paper's convention); may be NULL for types without nodes or
 *             without parameters
 *   U         device float32 [|V|][2][T] in reordered (sigma) order. Rows of processed nodes
 *             (positions >= K) are written; rows [0, K) are neither read nor written: input
 *             rows are read from S. The graph output is Y = U + step_ptr[N] * 2 * T, one row per
 *             output node in node order.
 *   ws        device workspace of >= grafx_workspace_bytes(sched, T, with_backward) bytes,
 *             256-byte aligned; a later grafx_render_backward needs the same workspace contents
 * Errors: GRAFX_E_ARG (null handle/pointers), GRAFX_E_SHAPE (T < 1, misaligned buffers, missing
 * parameter pointer), GRAFX_E_WORKSPACE, GRAFX_E_HIP. NaN/Inf in inputs propagate.
 */
grafx_status grafx_render(const grafx_schedule_t* sched, const void* dev_plan, int64_t T,
                          const float* S, const float* const* P, float* U, void* ws,
                          size_t ws_bytes, hipStream_t stream);

/*
 * grafx_render_noalloc -- grafx_render for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc. The same render
 * (same kernels, same bits) with the workspace taken from a static scratch array inside the
 * library instead of a caller buffer.
 *
 *   dev_plan, T, S, P, U, stream   exactly as for grafx_render
 * Scratch: one array of GRAFX_NOALLOC_SCRATCH_BYTES (32 MiB) per GPU, in the library's code
 * object; each GPU the library runs on holds it until the process ends. The first call on a
 * device (the device current on the calling thread, which must own `stream`) looks up the
 * array's address there; no call allocates or frees memory. A render whose forward workspace
 * (grafx_workspace_bytes with with_backward = 0) exceeds the scratch fails with
 * GRAFX_E_WORKSPACE before any device work: use grafx_render then. The call clears what must
 * start at zero (the dynamics chunk states and the error word) itself; everything else it
 * writes before reading.
 * Every call on a GPU shares that GPU's scratch, which keeps the last call's contents: two calls
 * whose device work overlaps on one GPU (different streams, or different threads without
 * ordering) race and give undefined results. The scratch is not a render workspace for
 * grafx_render_backward or grafx_workspace_error; a caller that needs the adjoint renders with
 * grafx_render into its own workspace. A caller that captures should make its first call on each
 * device outside capture (the address lookup is a runtime query, not stream work).
 * Errors: those of grafx_render (the workspace checks replaced by the size check above), and
 * GRAFX_E_HIP if the current device or the scratch address cannot be determined.
 */
#define GRAFX_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
grafx_status grafx_render_noalloc(const grafx_schedule_t* sched, const void* dev_plan, int64_t T,
                                  const float* S, const float* const* P, float* U,
                                  hipStream_t stream);

/*
 * grafx_render_backward -- adjoint of grafx_render (the backpropagation through the render that
 * gradient-descent matching needs, paper Sec. 4). Steps run in reverse order; each node's
 * output adjoint is gathered from the input adjoints of its successors, each node's input is
 * re-gathered from U and S, and the processor's adjoint writes the node's input adjoint and
 * its parameter-gradient partials; partials are reduced in a fixed order (deterministic).
 * Internal signals are recomputed from U; only the compressor's per-chunk envelope carries are
 * kept from the forward call (in `ws`).
 *
 *   P, S, U, T, dev_plan   exactly as passed to (and produced by) the preceding grafx_render
 *   ws       the workspace of that grafx_render call (sized with with_backward = 1)
 *   dY       device float32 [|V_N|][2][T], adjoint of the outputs
 *   dU       device float32 [|V|][2][T] scratch for the input adjoints (rows of processed
 *            nodes are written; rows [0, K) and output rows are not used)
 *   dS       device float32 [K][2][T] or NULL: adjoint of the sources
 *   dP       host array of GRAFX_NUM_TYPES device pointers or NULL; dP[t] (same layout as P[t])
 *            receives the parameter gradient (overwritten, not accumulated); a NULL entry skips
 *            that type. Delay phasors (re z, im z) receive 0 unless the delay-time surrogate is
 *            on (grafx_schedule_set_delay_surrogate).
 */
grafx_status grafx_render_backward(const grafx_schedule_t* sched, const void* dev_plan,
                                   int64_t T, const float* S, const float* const* P,
                                   const float* U, const float* dY, float* dU, float* dS,
                                   float* const* dP, void* ws, size_t ws_bytes,
                                   hipStream_t stream);

/*
 * Single steps of the two loops above, for callers that drive or time the loop themselves:
 * grafx_render_step runs the batched processor call of step `step` (1..N) only;
 * grafx_render_backward_step runs the adjoint of step `step` (1..N-1) only, leaving its
 * parameter-gradient partials in `ws` (the final reduction into dP happens in
 * grafx_render_backward). Preconditions: a complete grafx_render with the same parameters has
 * already run on `ws` (filter designs and envelope carries are there), and the rows the step
 * reads are current (earlier steps' outputs in U; later steps' input adjoints in dU).
 * Arguments and errors are those of grafx_render / grafx_render_backward, plus GRAFX_E_ARG for a
 * step out of range.
 */
grafx_status grafx_render_step(const grafx_schedule_t* sched, const void* dev_plan, int64_t T,
                               const float* S, const float* const* P, float* U, void* ws,
                               size_t ws_bytes, int32_t step, hipStream_t stream);
grafx_status grafx_render_backward_step(const grafx_schedule_t* sched, const void* dev_plan,
                                        int64_t T, const float* S, const float* const* P,
                                        const float* U, const float* dY, float* dU, void* ws,
                                        size_t ws_bytes, int32_t step, hipStream_t stream);

/*
 * Settings of a schedule. The tuning knobs are chosen by a caller-side autotuner from measured
 * step times (the paper picks its batching per graph on the host, Sec. 2 "Implementation
 * details"; these settings pick launch shapes the same way). A tuning knob changes which threads
 * and blocks share the work, hence the grouping of the per-block parameter-gradient partial sums
 * (results stay within the parity tolerances; each setting is deterministic), never the
 * per-sample arithmetic or the workspace size.
 *   GRAFX_TUNE_POINTWISE_UNROLL: 1024-sample parts per block of the pointwise kernels (mix, out,
 *     gain_pan, imager, tanh): 1 (default), 2 or 4.
 *   GRAFX_TUNE_EQ_ORDER: order of the EQ kernels' blocks: 0 (default) maps the tiles of one node
 *     onto one XCD (neighbouring tiles share their halo through its L2), 1 keeps the hardware's
 *     round-robin order (another XCD then fetches the halo again). Same bits either way.
 *   GRAFX_TUNE_DYN_ORDER: order of the dynamics kernels' blocks (compressor, noisegate,
 *     compressor_ar): 0 issues a node's chunks contiguously, 1 interleaves the step's nodes block
 *     by block, so that a chunk's predecessors have usually published by the time it starts;
 *     2 (default) interleaves a launch of at least 4096 blocks (several rounds of resident
 *     blocks) and keeps a smaller one contiguous. Chunks are still taken in ticket order per
 *     node: same bits.
 *   GRAFX_TUNE_TAP_TILES: time tiles (2048 samples) per block of the delay's tap-gradient pass:
 *     4, 8 or 16 (default); sets the grouping of the tap-gradient partial sums.
 * Two settings bound the iterative parts of the dynamics kernels instead:
 *   GRAFX_TUNE_AR_MAX_PASSES: branch-pattern passes of the attack/release compressor's forward
 *     (Eq. 8 with distinct coefficients) before a chunk that has not settled falls back to the
 *     serial recursion, 1..16 (default 16). Every value gives the exact recursion; a small value
 *     sends more chunks to the fallback.
 *   GRAFX_TUNE_WAIT_POLLS: polls of a published chunk state that a dynamics block makes before
 *     it gives up waiting, 0..2^30 (default 2^24, far beyond any wait a completing launch
 *     needs). A wait that gives up sets bit 0 of the workspace's error word
 *     (grafx_workspace_error) and poisons its result with NaN; the kernel still exits normally.
 *     0 makes every wait give up at once (a test of that path from the host).
 * grafx_schedule_set_tuning: E_ARG for a NULL schedule, an unknown knob or a value out of range.
 * A setting applies to every later call with the schedule; calls that overlap with a change on
 * another thread are not synchronised with it. A HIP graph captured from render calls keeps the
 * settings in force at capture time.
 */
enum {
  GRAFX_TUNE_POINTWISE_UNROLL = 0, GRAFX_TUNE_AR_MAX_PASSES = 1, GRAFX_TUNE_WAIT_POLLS = 2,
  GRAFX_TUNE_EQ_ORDER = 3, GRAFX_TUNE_DYN_ORDER = 4, GRAFX_TUNE_TAP_TILES = 5
};
grafx_status grafx_schedule_set_tuning(grafx_schedule_t* sched, int32_t knob, int32_t value);
grafx_status grafx_schedule_get_tuning(const grafx_schedule_t* sched, int32_t knob,
                                       int32_t* value);

/*
 * grafx_schedule_set_reverb_noise -- the fixed noise realisation of the reverb (paper Sec. 3
 * "Reverb": the impulse response is a noise signal shaped by the mask of Eq. 7 in the STFT
 * domain, then turned from mid/side into left/right).
 *
 *   noise   device float32 [2][length]: the mid noise, then the side noise; every reverb node of
 *           the schedule uses it. Borrowed, not copied: it must stay valid and unchanged while
 *           any render or adjoint that uses the schedule runs. NULL (with length 0) clears it.
 *   length  samples per signal, 1..GRAFX_REVERB_MAX_LEN; it is also the length of every reverb
 *           node's FIR (2 s, 88200 samples, in the paper) and enters the workspace size, so set
 *           it before grafx_workspace_bytes.
 * Renders of a graph with reverb nodes fail with GRAFX_E_ARG while no noise is set.
 * Errors: GRAFX_E_ARG (NULL schedule, NULL noise with a non-zero length), GRAFX_E_SHAPE (length
 * out of range, noise not 4-byte aligned).
 */
#define GRAFX_REVERB_MAX_LEN ((int64_t)1 << 22)
grafx_status grafx_schedule_set_reverb_noise(grafx_schedule_t* sched, const float* noise,
                                            int64_t length);

/*
 * grafx_schedule_set_delay_surrogate -- the gradient of the delay times (paper Sec. 3 "Multitap
 * delay", Eq. 15), for both delay types (delay, delay_long). With enable = 0 (the default)
 * grafx_render_backward writes 0 to every delay phasor entry (re z, im z). With enable = 1 it writes the straight-through gradient of the
 * surrogate: the render keeps the exact integer delay of each 100 ms slot, and the phasor z of the
 * slot gets the gradient that the render would have if the slot's unit impulse were the real part
 * of s[n] = (1/4410) sum_{k=0}^{4409} z^k exp(2 pi i k n / 4410), n = 0..4409 lags from the slot's
 * start (the unit impulse at the integer delay when z lies on the unit circle at that delay).
 * The paper's per-delay gradient normalisation and its unit-circle regulariser belong to the
 * optimiser and are not applied here. The setting enters the adjoint's workspace size (spectra of
 * every delay node's input and output adjoint), so set it before grafx_workspace_bytes.
 * Errors: GRAFX_E_ARG (NULL schedule, enable not 0 or 1).
 */
grafx_status grafx_schedule_set_delay_surrogate(grafx_schedule_t* sched, int32_t enable);

/*
 * grafx_delay_phasor_regularise -- the optimiser-side treatment of the delay-time gradients that
 * the paper applies with the surrogate (Sec. 3 "Multitap delay": each delay's gradient is
 * normalised and z is regularised towards the unit circle; the paper gives neither the norm nor
 * the regulariser, so this is one reading). For every phasor of n nodes of one delay type, in
 * place on dP: the pair (dL/dRe z, dL/dIm z) is scaled to unit length (a zero pair stays zero),
 * then the gradient of weight * (|z| - 1)^2, i.e. 2 weight (|z| - 1) z / |z| (zero at z = 0), is
 * added. Log-magnitude entries are not touched.
 *   delay_type  GRAFX_DELAY (rows of 220) or GRAFX_DELAY_LONG (rows of 880)
 *   n           number of rows (>= 0)
 *   P, dP       device float32 [n][row]: the parameters and their gradient (as written by
 *               grafx_render_backward with the surrogate on)
 *   weight      regulariser weight, finite and >= 0
 * Errors: GRAFX_E_TYPE (other type), GRAFX_E_SHAPE (n < 0, misaligned), GRAFX_E_ARG (NULL
 * buffers with n > 0, bad weight), GRAFX_E_HIP.
 */
grafx_status grafx_delay_phasor_regularise(int32_t delay_type, int32_t n, const float* P,
                                           float* dP, float weight, hipStream_t stream);

/*
 * grafx_workspace_error -- the error word of the dynamics kernels (compressor, noisegate,
 * compressor_ar; the chunked scan of Eq. 8) in a render workspace: enqueues on `stream` a copy of
 * the 32-bit word into `word` (host or device memory; read it after the stream has completed).
 *   bit 0  a chunk wait gave up (GRAFX_TUNE_WAIT_POLLS): the affected outputs are NaN
 *   bit 1  a dynamics kernel found its chunk tickets not reset and did nothing (only possible if
 *          a caller ran kernels on a workspace outside the render calls' order)
 * grafx_render and grafx_render_step clear the word before their first dynamics launch;
 * grafx_render_backward and grafx_render_backward_step add their own bits to it, so after a
 * render and its adjoint the word reports both. A schedule without dynamics nodes reports 0.
 *   T, ws, ws_bytes   as passed to the render calls (ws_bytes >= the forward workspace size)
 * Errors: GRAFX_E_ARG (NULL argument), GRAFX_E_SHAPE (T out of range, misaligned workspace),
 * GRAFX_E_WORKSPACE (workspace too small), GRAFX_E_HIP (the copy could not be enqueued).
 */
grafx_status grafx_workspace_error(const grafx_schedule_t* sched, int64_t T, const void* ws,
                                   size_t ws_bytes, uint32_t* word, hipStream_t stream);

/*
 * Multi-resolution STFT loss between two sets of stereo signals (the loss of the paper's
 * gradient-descent mixing application, Sec. 4): resolutions 512, 1024 and 2048, hop r/4,
 * periodic Hann window, frames that fit inside [0, T), magnitudes sqrt(|X|^2 + 1e-8);
 * L = (1/3) sum_r (||S_y - S_t||_F / ||S_t||_F + mean |ln S_y - ln S_t|).
 *
 *   rows       number of stereo rows in Y and target (e.g. the output nodes)
 *   Y, target  device float32 [rows][2][T]
 *   loss       device float32 scalar (written)
 *   ws         device workspace of >= grafx_mrstft_workspace_bytes(rows, T) bytes; the
 *              backward call must see the contents left by the forward call
 * grafx_mrstft_backward writes dY = dloss * dL/dY (overwritten) where dloss is a device float32
 * scalar (the upstream gradient).
 */
grafx_status grafx_mrstft_workspace_bytes(int32_t rows, int64_t T, size_t* bytes);
grafx_status grafx_mrstft_loss(int32_t rows, int64_t T, const float* Y, const float* target,
                               float* loss, void* ws, size_t ws_bytes, hipStream_t stream);
grafx_status grafx_mrstft_backward(int32_t rows, int64_t T, const float* Y,
                                   const float* target, const float* dloss, float* dY, void* ws,
                                   size_t ws_bytes, hipStream_t stream);

/*
 * Learned parameter initialiser for the gradient-descent mixing application (Sec. 4): a
 * convolutional encoder predicts the normalised parameters of a track's gain_pan -> eq ->
 * compressor chain from the log-mel features of the dry track and of the target mix.
 *
 * grafx_logmel: features [n_signals][128][F] (device float32, overwritten) of stereo signals
 *   [n_signals][2][T] (device float32), F = (T - 1024) / 256 + 1: mono (l + r) / 2, frames of
 *   1024 samples at hop 256 inside [0, T), periodic Hann window, power spectrum, 128 triangular
 *   filters on the HTK mel scale (130 edges evenly spaced in mel over [0, 22050] Hz, peak 1),
 *   feature (ln(E + 1e-6) + 5) / 5. E_SHAPE unless 1024 <= T < 2^29.
 * grafx_encoder_gather: encoder input x [batch][256][F]: rows 0..127 of sample b are
 *   dry_features[dry[b]], rows 128..255 mix_features[mix[b]] (feature tables [n][128][F]; int32
 *   device index arrays of length batch, each index below its table's n, not checked); if
 *   label_table ([n_dry][11]) is not NULL, labels[b] = label_table[dry[b]] as well.
 * grafx_encoder_sizes: number of float32 weights (one flat buffer: per layer l = 1..6 the
 *   weights [64][C_in][5] (C_in = 256, then 64) and the bias [64], then the head [11][64] and
 *   its bias [11]), of activation floats and of backward scratch floats for a batch of
 *   `batch` inputs of `frames` frames (1 <= batch, frames <= 2^20, else E_SHAPE).
 * grafx_encoder_forward: six convolutions (kernel 5, stride 2, zero padding 2, bias, ReLU), mean
 *   over frames, linear head, sigmoid: out [batch][11] in (0, 1) (device, overwritten). acts
 *   (device, act_floats) receives the activations the backward needs. bf16 != 0 runs the
 *   convolutions on the matrix cores in bfloat16 with float32 accumulation (inference).
 * grafx_encoder_backward: mean squared error against labels [batch][11] (device) into *loss
 *   (device scalar, may be NULL) and its gradient with respect to every weight into dweights
 *   (device, n_weights floats, overwritten); x, weights, acts and out as left by a float32
 *   forward call; grads is scratch of grad_floats. Fixed summation orders: bit-reproducible.
 * grafx_adam: one Adam step over n float32 values in place: m = b1 m + (1 - b1) g,
 *   v = b2 v + (1 - b2) g^2, p -= lr s (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps)
 *   with s = lr_scale[i] (device, n floats) or 1 when lr_scale is NULL (a zero scale freezes a
 *   value); step >= 1 counts from 1 (E_ARG otherwise).
 * grafx_encoder_params: parameter rows of the chain from normalised outputs [batch][11]:
 *   gain_pan [batch][2] (dB [-12, 6] per channel as natural-log gains), eq [batch][1024] (six
 *   band gains [-12, 12] dB at 20 * 1000^((b + 0.5) / 6) Hz, linear in log-frequency over bins
 *   k fs / 2047 Hz, constant beyond the outer bands), compressor [batch][4] (alpha from a time
 *   constant of [1, 100] ms, threshold [-30, -10] dB, knee 3 dB, ratio [2, 8]).
 * All pointers are device pointers except the size outputs; every call only enqueues work.
 */
grafx_status grafx_logmel(int32_t n_signals, int64_t T, const float* signals, float* features,
                          hipStream_t stream);
grafx_status grafx_encoder_gather(int32_t batch, int32_t frames, const float* dry_features,
                                  const int32_t* dry, const float* mix_features,
                                  const int32_t* mix, const float* label_table, float* labels,
                                  float* x, hipStream_t stream);
grafx_status grafx_encoder_sizes(int32_t batch, int32_t frames, size_t* n_weights,
                                 size_t* act_floats, size_t* grad_floats);
grafx_status grafx_encoder_forward(int32_t batch, int32_t frames, const float* x,
                                   const float* weights, int32_t bf16, float* acts, float* out,
                                   hipStream_t stream);
grafx_status grafx_encoder_backward(int32_t batch, int32_t frames, const float* x,
                                    const float* weights, const float* acts, const float* out,
                                    const float* labels, float* loss, float* dweights,
                                    float* grads, hipStream_t stream);
grafx_status grafx_adam(int64_t n, float* p, const float* g, float* m, float* v,
                        const float* lr_scale, int32_t step, float lr, float beta1, float beta2,
                        float eps, hipStream_t stream);
grafx_status grafx_encoder_params(int32_t batch, const float* out, float* gain_pan, float* eq,
                                  float* comp, hipStream_t stream);

/*
 * grafx_last_error -- message of the last failed call on the calling thread ("" if the last
 * call succeeded). Every entry point clears it on entry and sets it with the status it returns,
 * so the message always names the check that failed (the error model of the boundary; the paper
 * has no error model of its own). The string stays valid until the thread's next call.
 */
const char* grafx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GRAFX_H_ */
