// Host scheduler: type-homogeneous, causal, maximal-subset schedules of an audio processing graph
// and the reordered read/write index lists (paper Sec. 2 "Batched processing", "Type scheduling",
// "Implementation details"; Algorithm 1, preprocessing).
//
// Computed-node sets are dense bitsets; the beam and optimal searches deduplicate children by set
// (keeping the lexicographically smallest type string) and rank them by (more nodes computed,
// smaller string). Every tie-break is fixed, so the schedule is a pure function of the graph.
//
// The preprocessing runs on the CPU, off the GPU's path (Sec. 2, "Implementation details"), and
// a large search uses several host threads: the states of one search depth are split into
// contiguous slices, each thread expands its slice, and the children are merged in the serial
// order (state by state, types ascending), so the result does not depend on the thread count.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "grafx_internal.h"

namespace grafx {

namespace {
thread_local std::string g_error;
}

grafx_status fail(grafx_status code, const std::string& msg) {
  g_error = msg;
  return code;
}

void clear_error() { g_error.clear(); }

namespace {

using Word = uint64_t;

struct Bits {
  std::vector<Word> w;
  explicit Bits(size_t n = 0) : w((n + 63) / 64, 0) {}
  bool get(int i) const { return (w[i >> 6] >> (i & 63)) & 1u; }
  void set(int i) { w[i >> 6] |= Word(1) << (i & 63); }
  void or_with(const Bits& o) {
    for (size_t k = 0; k < w.size(); ++k) w[k] |= o.w[k];
  }
  int count() const {
    int c = 0;
    for (Word x : w) c += __builtin_popcountll(x);
    return c;
  }
  bool operator==(const Bits& o) const { return w == o.w; }
};

struct BitsHash {
  size_t operator()(const Bits& b) const {
    uint64_t h = 0x9E3779B97F4A7C15ull;
    for (Word x : b.w) {
      h ^= x + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
      h *= 0xBF58476D1CE4E5B9ull;
    }
    return static_cast<size_t>(h ^ (h >> 31));
  }
};

struct Graph {
  int V = 0;
  std::vector<int32_t> type;
  std::vector<int32_t> pred_ptr, pred;  // unique predecessors per node
  std::vector<int32_t> proc;            // processing nodes (not in/out), ascending id
  Bits start, full;
};

// Ready processing nodes of each type for the computed set C (nodes not in C whose
// predecessors are all in C). by_type[t] lists them in ascending id.
void ready_by_type(const Graph& g, const Bits& C, std::vector<std::vector<int32_t>>& by_type) {
  for (auto& v : by_type) v.clear();
  for (int32_t v : g.proc) {
    if (C.get(v)) continue;
    bool ok = true;
    for (int32_t k = g.pred_ptr[v]; k < g.pred_ptr[v + 1]; ++k)
      if (!C.get(g.pred[k])) { ok = false; break; }
    if (ok) by_type[g.type[v]].push_back(v);
  }
}

struct State {
  Bits C;
  std::vector<int8_t> s;
  int pop = 0;
};

std::atomic<int> g_threads{0};  // 0: default

int search_threads() {
  const int n = g_threads.load(std::memory_order_relaxed);
  if (n > 0) return n;
  const int hw = static_cast<int>(std::thread::hardware_concurrency());
  return std::max(1, std::min(hw, 16));
}

// Every child of states[a, b): for each state in order, one child per non-empty type in
// ascending type order.
void expand(const Graph& g, const std::vector<State>& states, size_t a, size_t b,
            std::vector<State>& out) {
  std::vector<std::vector<int32_t>> by(kNumTypes);
  for (size_t i = a; i < b; ++i) {
    const State& st = states[i];
    ready_by_type(g, st.C, by);
    for (int t = 0; t < kNumTypes; ++t) {
      if (by[t].empty()) continue;
      State ch;
      ch.C = st.C;
      for (int32_t v : by[t]) ch.C.set(v);
      ch.s = st.s;
      ch.s.push_back(static_cast<int8_t>(t));
      ch.pop = st.pop + static_cast<int>(by[t].size());
      out.push_back(std::move(ch));
    }
  }
}

// Work (states x processing nodes) below which one depth is expanded on the calling thread.
constexpr size_t kParallelWork = size_t(1) << 16;

// Threads kept for one search: run(f) calls f(0) on the calling thread and f(1..n-1) on the
// pool's threads, and returns when every call has returned.
class SearchPool {
 public:
  explicit SearchPool(int n) : n_(n) {
    for (int k = 1; k < n; ++k) threads_.emplace_back([this, k] { work(k); });
  }
  ~SearchPool() {
    {
      std::lock_guard<std::mutex> lock(m_);
      stop_ = true;
    }
    go_.notify_all();
    for (auto& t : threads_) t.join();
  }
  int size() const { return n_; }
  void run(const std::function<void(int)>& f) {
    {
      std::lock_guard<std::mutex> lock(m_);
      job_ = f;
      pending_ = n_ - 1;
      ++generation_;
    }
    go_.notify_all();
    f(0);
    std::unique_lock<std::mutex> lock(m_);
    done_.wait(lock, [&] { return pending_ == 0; });
  }

 private:
  void work(int k) {
    uint64_t seen = 0;
    for (;;) {
      std::function<void(int)> job;
      {
        std::unique_lock<std::mutex> lock(m_);
        go_.wait(lock, [&] { return stop_ || generation_ != seen; });
        if (stop_) return;
        seen = generation_;
        job = job_;
      }
      job(k);
      std::lock_guard<std::mutex> lock(m_);
      if (--pending_ == 0) done_.notify_one();
    }
  }
  const int n_;
  std::vector<std::thread> threads_;
  std::mutex m_;
  std::condition_variable go_, done_;
  std::function<void(int)> job_;
  int pending_ = 0;
  uint64_t generation_ = 0;
  bool stop_ = false;
};

grafx_status search_one_by_one(const Graph& g, std::vector<std::vector<int32_t>>& steps) {
  Bits C = g.start;
  std::vector<std::vector<int32_t>> by(kNumTypes);
  const int n_proc = static_cast<int>(g.proc.size());
  for (int it = 0; it < n_proc; ++it) {
    ready_by_type(g, C, by);
    int32_t best = -1;
    for (int t = 0; t < kNumTypes; ++t)
      if (!by[t].empty() && (best < 0 || by[t][0] < best)) best = by[t][0];
    if (best < 0) return fail(GRAFX_E_GRAPH, "no ready node (internal)");
    steps.push_back({best});
    C.set(best);
  }
  return GRAFX_OK;
}

grafx_status search_greedy(const Graph& g, std::vector<int8_t>& types) {
  Bits C = g.start;
  std::vector<std::vector<int32_t>> by(kNumTypes);
  while (!(C == g.full)) {
    ready_by_type(g, C, by);
    int best = -1;
    for (int t = 0; t < kNumTypes; ++t)
      if (!by[t].empty() && (best < 0 || by[t].size() > by[best].size())) best = t;
    if (best < 0) return fail(GRAFX_E_GRAPH, "no ready node (internal)");
    for (int32_t v : by[best]) C.set(v);
    types.push_back(static_cast<int8_t>(best));
  }
  return GRAFX_OK;
}

// Beam search over maximal-subset type strings; width < 0 means unbounded (optimal).
grafx_status search_beam(const Graph& g, int64_t width, int64_t state_limit,
                         std::vector<int8_t>& types) {
  std::vector<State> states(1);
  states[0].C = g.start;
  states[0].pop = g.start.count();
  const int full_pop = g.full.count();
  std::unique_ptr<SearchPool> pool;  // created at the first depth large enough to split
  for (;;) {
    const State* best_done = nullptr;
    for (const State& st : states)
      if (st.pop == full_pop && st.C == g.full)
        if (!best_done || st.s < best_done->s) best_done = &st;
    if (best_done) {
      types = best_done->s;
      return GRAFX_OK;
    }
    // expansion (in slices on several threads when the depth is large), then the merge in the
    // serial order with deduplication by computed set
    const size_t ns = states.size();
    if (!pool && ns > 1 && ns * g.proc.size() >= kParallelWork && search_threads() > 1)
      pool = std::make_unique<SearchPool>(search_threads());
    const int nt = pool && ns * g.proc.size() >= kParallelWork
                       ? static_cast<int>(std::min<size_t>(ns, pool->size()))
                       : 1;
    std::vector<std::vector<State>> part(nt);
    if (nt == 1) {
      expand(g, states, 0, ns, part[0]);
    } else {
      pool->run([&](int k) {
        if (k < nt) expand(g, states, ns * k / nt, ns * (k + 1) / nt, part[k]);
      });
    }
    std::vector<State> children;
    std::unordered_map<Bits, size_t, BitsHash> index;
    for (auto& pk : part)
      for (State& ch : pk) {
        auto it = index.find(ch.C);
        if (it == index.end()) {
          index.emplace(ch.C, children.size());
          children.push_back(std::move(ch));
        } else if (ch.s < children[it->second].s) {
          children[it->second].s = std::move(ch.s);
        }
      }
    if (children.empty()) return fail(GRAFX_E_GRAPH, "schedule search stalled (internal)");
    std::sort(children.begin(), children.end(), [](const State& a, const State& b) {
      if (a.pop != b.pop) return a.pop > b.pop;
      return a.s < b.s;
    });
    if (width < 0) {
      if (static_cast<int64_t>(children.size()) > state_limit)
        return fail(GRAFX_E_LIMIT, "optimal schedule search exceeded the state limit");
    } else if (static_cast<int64_t>(children.size()) > width) {
      children.resize(static_cast<size_t>(width));
    }
    states = std::move(children);
  }
}

grafx_status replay(const Graph& g, const std::vector<int8_t>& types,
                    std::vector<std::vector<int32_t>>& steps) {
  Bits C = g.start;
  std::vector<std::vector<int32_t>> by(kNumTypes);
  for (int8_t t : types) {
    ready_by_type(g, C, by);
    if (by[t].empty()) return fail(GRAFX_E_GRAPH, "type string replay failed (internal)");
    for (int32_t v : by[t]) C.set(v);
    steps.push_back(by[t]);
  }
  return GRAFX_OK;
}

}  // namespace
}  // namespace grafx

namespace grafx {
namespace {

// Packed host image of the device plan: int32 sections on 64-element boundaries.
void build_plan(grafx_schedule_t* h) {
  const size_t V = h->V, E = h->E;
  PlanLayout& L = h->layout;
  size_t off = 0;
  auto take = [&](size_t n) { size_t o = off; off = align_up(off + n, 64); return o; };
  L.in_ptr = take(V + 1);
  L.in_src = take(E);
  L.out_ptr = take(V + 1);
  L.out_dst = take(E);
  L.param_row = take(V);
  L.len = take(h->node_len.size());
  L.total = off;
  h->plan.assign(L.total, 0);
  std::copy(h->in_ptr.begin(), h->in_ptr.end(), h->plan.begin() + L.in_ptr);
  std::copy(h->in_src.begin(), h->in_src.end(), h->plan.begin() + L.in_src);
  std::copy(h->out_ptr.begin(), h->out_ptr.end(), h->plan.begin() + L.out_ptr);
  std::copy(h->out_dst.begin(), h->out_dst.end(), h->plan.begin() + L.out_dst);
  std::copy(h->param_row.begin(), h->param_row.end(), h->plan.begin() + L.param_row);
  std::copy(h->node_len.begin(), h->node_len.end(), h->plan.begin() + L.len);
}

}  // namespace
}  // namespace grafx

using namespace grafx;

extern "C" {

const char* grafx_last_error(void) { return g_error.c_str(); }

int32_t grafx_set_schedule_threads(int32_t n) {
  if (n < 0) return g_threads.load();
  return g_threads.exchange(n);
}

grafx_status grafx_schedule(int32_t num_nodes, const int32_t* node_type, int32_t num_edges,
                            const int32_t* edge_src, const int32_t* edge_dst,
                            const int32_t* edge_type, int32_t method, int32_t beam_width,
                            int64_t state_limit, grafx_schedule_t** out) {
  clear_error();
  if (!out) return fail(GRAFX_E_ARG, "out is NULL");
  *out = nullptr;
  if (num_nodes < 1) return fail(GRAFX_E_ARG, "graph has no nodes");
  if (!node_type) return fail(GRAFX_E_ARG, "node_type is NULL");
  if (num_edges < 0) return fail(GRAFX_E_ARG, "num_edges is negative");
  if (num_edges > 0 && (!edge_src || !edge_dst)) return fail(GRAFX_E_ARG, "edge list is NULL");
  const int V = num_nodes, E = num_edges;
  for (int v = 0; v < V; ++v)
    if (node_type[v] < 0 || node_type[v] >= kNumTypes)
      return fail(GRAFX_E_TYPE, "node " + std::to_string(v) + " has an unknown type");
  for (int e = 0; e < E; ++e)
    if (edge_src[e] < 0 || edge_src[e] >= V || edge_dst[e] < 0 || edge_dst[e] >= V)
      return fail(GRAFX_E_GRAPH, "edge " + std::to_string(e) + " references a missing node");
  if (edge_type)
    for (int e = 0; e < 2 * E; ++e)
      if (edge_type[e] != 0)
        return fail(GRAFX_E_TYPE, "multi-port edge types are not supported (SISO only)");
  for (int e = 0; e < E; ++e) {
    if (node_type[edge_dst[e]] == GRAFX_IN)
      return fail(GRAFX_E_GRAPH, "edge " + std::to_string(e) + " enters an input node");
    if (node_type[edge_src[e]] == GRAFX_OUT)
      return fail(GRAFX_E_GRAPH, "edge " + std::to_string(e) + " leaves an output node");
  }
  bool has_out = false;
  for (int v = 0; v < V; ++v) has_out |= node_type[v] == GRAFX_OUT;
  if (!has_out) return fail(GRAFX_E_GRAPH, "graph has no output node");
  {  // cycle check (Kahn)
    std::vector<int32_t> indeg(V, 0), sptr(V + 1, 0), sl(E);
    for (int e = 0; e < E; ++e) { indeg[edge_dst[e]]++; sptr[edge_src[e] + 1]++; }
    for (int v = 0; v < V; ++v) sptr[v + 1] += sptr[v];
    std::vector<int32_t> fillp(sptr.begin(), sptr.end() - 1);
    for (int e = 0; e < E; ++e) sl[fillp[edge_src[e]]++] = edge_dst[e];
    std::vector<int32_t> stack;
    for (int v = 0; v < V; ++v) if (indeg[v] == 0) stack.push_back(v);
    int seen = 0;
    while (!stack.empty()) {
      int v = stack.back(); stack.pop_back(); ++seen;
      for (int k = sptr[v]; k < sptr[v + 1]; ++k) if (--indeg[sl[k]] == 0) stack.push_back(sl[k]);
    }
    if (seen != V) return fail(GRAFX_E_CYCLE, "graph has a cycle");
  }
  if (method < GRAFX_SCHED_ONE_BY_ONE || method > GRAFX_SCHED_OPTIMAL)
    return fail(GRAFX_E_ARG, "unknown schedule method");
  if (method == GRAFX_SCHED_BEAM && beam_width < 1)
    return fail(GRAFX_E_ARG, "beam width must be positive");
  if (method == GRAFX_SCHED_OPTIMAL && state_limit < 1)
    return fail(GRAFX_E_ARG, "state limit must be positive");

  Graph g;
  g.V = V;
  g.type.assign(node_type, node_type + V);
  {  // unique predecessors
    std::vector<std::vector<int32_t>> pl(V);
    for (int e = 0; e < E; ++e) pl[edge_dst[e]].push_back(edge_src[e]);
    g.pred_ptr.assign(V + 1, 0);
    for (int v = 0; v < V; ++v) {
      auto& p = pl[v];
      std::sort(p.begin(), p.end());
      p.erase(std::unique(p.begin(), p.end()), p.end());
      g.pred_ptr[v + 1] = g.pred_ptr[v] + static_cast<int32_t>(p.size());
      g.pred.insert(g.pred.end(), p.begin(), p.end());
    }
  }
  g.start = Bits(V);
  g.full = Bits(V);
  for (int v = 0; v < V; ++v) {
    if (g.type[v] == GRAFX_IN) { g.start.set(v); g.full.set(v); }
    else if (g.type[v] != GRAFX_OUT) { g.proc.push_back(v); g.full.set(v); }
  }


  std::vector<std::vector<int32_t>> steps;
  {
    std::vector<int32_t> ins;
    for (int v = 0; v < V; ++v) if (g.type[v] == GRAFX_IN) ins.push_back(v);
    steps.push_back(ins);
  }
  grafx_status st = GRAFX_OK;
  if (method == GRAFX_SCHED_ONE_BY_ONE) {
    st = search_one_by_one(g, steps);
  } else {
    std::vector<int8_t> types;
    if (method == GRAFX_SCHED_GREEDY) st = search_greedy(g, types);
    else if (method == GRAFX_SCHED_BEAM) st = search_beam(g, beam_width, 0, types);
    else st = search_beam(g, -1, state_limit, types);
    if (st == GRAFX_OK) st = replay(g, types, steps);
  }
  if (st != GRAFX_OK) return st;
  {
    std::vector<int32_t> outs;
    for (int v = 0; v < V; ++v) if (g.type[v] == GRAFX_OUT) outs.push_back(v);
    steps.push_back(outs);
  }

  auto* h = new grafx_schedule_t();
  h->V = V;
  h->E = E;
  h->N = static_cast<int32_t>(steps.size()) - 1;
  h->node_type = g.type;
  for (int v = 0; v < V; ++v) h->type_count[g.type[v]]++;
  h->K = h->type_count[GRAFX_IN];
  h->n_out = h->type_count[GRAFX_OUT];
  // reorder by (step, original id): steps already list their nodes in ascending id
  std::vector<int32_t> pos(V);
  h->step_ptr.push_back(0);
  for (size_t n = 0; n < steps.size(); ++n) {
    h->step_type.push_back(n == 0 ? GRAFX_IN
                                  : (n + 1 == steps.size() ? GRAFX_OUT : g.type[steps[n][0]]));
    for (int32_t v : steps[n]) { pos[v] = static_cast<int32_t>(h->perm.size()); h->perm.push_back(v); }
    h->step_ptr.push_back(static_cast<int32_t>(h->perm.size()));
  }
  // in/out CSR in reordered order, lists in original edge order
  std::vector<int32_t> in_cnt(V, 0), out_cnt(V, 0);
  for (int e = 0; e < E; ++e) { in_cnt[pos[edge_dst[e]]]++; out_cnt[pos[edge_src[e]]]++; }
  h->in_ptr.assign(V + 1, 0);
  h->out_ptr.assign(V + 1, 0);
  for (int i = 0; i < V; ++i) {
    h->in_ptr[i + 1] = h->in_ptr[i] + in_cnt[i];
    h->out_ptr[i + 1] = h->out_ptr[i] + out_cnt[i];
  }
  h->in_src.assign(E, 0);
  h->out_dst.assign(E, 0);
  {
    std::vector<int32_t> fi(h->in_ptr.begin(), h->in_ptr.end() - 1);
    std::vector<int32_t> fo(h->out_ptr.begin(), h->out_ptr.end() - 1);
    for (int e = 0; e < E; ++e) {
      const int32_t s = pos[edge_src[e]], d = pos[edge_dst[e]];
      h->in_src[fi[d]++] = s;
      h->out_dst[fo[s]++] = d;
    }
  }
  {
    std::vector<int32_t> row_of(V), seen(kNumTypes, 0);
    for (int v = 0; v < V; ++v) row_of[v] = seen[g.type[v]]++;
    h->param_row.resize(V);
    for (int i = 0; i < V; ++i) h->param_row[i] = row_of[h->perm[i]];
  }
  build_plan(h);
  *out = h;
  return GRAFX_OK;
}

grafx_status grafx_schedule_with_lengths(int32_t num_nodes, const int32_t* node_type,
                                         int32_t num_edges, const int32_t* edge_src,
                                         const int32_t* edge_dst, const int32_t* edge_type,
                                         const int32_t* node_len, int32_t method,
                                         int32_t beam_width, int64_t state_limit,
                                         grafx_schedule_t** out) {
  clear_error();
  if (!out) return fail(GRAFX_E_ARG, "out is NULL");
  *out = nullptr;
  if (!node_len) return fail(GRAFX_E_ARG, "node_len is NULL");
  if (!node_type) return fail(GRAFX_E_ARG, "node_type is NULL");
  if (num_edges > 0 && (!edge_src || !edge_dst)) return fail(GRAFX_E_ARG, "edge arrays are NULL");
  for (int32_t v = 0; v < num_nodes; ++v)
    if (node_len[v] < 1 || node_len[v] >= (1 << 29))
      return fail(GRAFX_E_SHAPE, "node " + std::to_string(v) + ": length must be in [1, 2^29)");
  for (int32_t e = 0; e < num_edges; ++e) {
    const int32_t a = edge_src[e], b = edge_dst[e];
    if (a < 0 || a >= num_nodes || b < 0 || b >= num_nodes) continue;  // grafx_schedule rejects
    if (node_len[a] != node_len[b])
      return fail(GRAFX_E_SHAPE, "edge " + std::to_string(e) +
                                     " joins nodes of different lengths (every connected graph "
                                     "has one length)");
  }
  grafx_schedule_t* h = nullptr;
  const grafx_status st = grafx_schedule(num_nodes, node_type, num_edges, edge_src, edge_dst,
                                         edge_type, method, beam_width, state_limit, &h);
  if (st != GRAFX_OK) return st;
  h->node_len.resize(h->V);
  h->max_len = 0;
  h->len4 = true;
  for (int i = 0; i < h->V; ++i) {
    const int32_t n = node_len[h->perm[i]];
    h->node_len[i] = n;
    h->max_len = std::max(h->max_len, n);
    h->len4 = h->len4 && (n % 4 == 0);
  }
  build_plan(h);
  *out = h;
  return GRAFX_OK;
}

void grafx_schedule_free(grafx_schedule_t* sched) { delete sched; }

grafx_status grafx_schedule_query(const grafx_schedule_t* h, grafx_schedule_sizes* out) {
  clear_error();
  if (!h || !out) return fail(GRAFX_E_ARG, "NULL argument");
  out->num_nodes = h->V;
  out->num_edges = h->E;
  out->num_steps = h->N;
  out->num_inputs = h->K;
  out->num_outputs = h->n_out;
  for (int t = 0; t < kNumTypes; ++t) out->type_count[t] = h->type_count[t];
  out->plan_bytes = static_cast<int64_t>(h->layout.total * sizeof(int32_t));
  out->max_len = h->max_len;
  return GRAFX_OK;
}

grafx_status grafx_schedule_export(const grafx_schedule_t* h, int32_t* step_type,
                                   int32_t* step_ptr, int32_t* perm, int32_t* in_ptr,
                                   int32_t* in_src, int32_t* out_ptr, int32_t* out_dst,
                                   int32_t* param_row) {
  clear_error();
  if (!h) return fail(GRAFX_E_ARG, "NULL schedule");
  auto put = [](const std::vector<int32_t>& v, int32_t* dst) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(int32_t));
  };
  put(h->step_type, step_type);
  put(h->step_ptr, step_ptr);
  put(h->perm, perm);
  put(h->in_ptr, in_ptr);
  put(h->in_src, in_src);
  put(h->out_ptr, out_ptr);
  put(h->out_dst, out_dst);
  put(h->param_row, param_row);
  return GRAFX_OK;
}

}  // extern "C"
