// C-ABI entry points of libsimrank and the host orchestration behind them.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <unordered_map>
#include <vector>

#include "hostgraph.h"
#include "kernels.h"
#include "simrank.h"

using namespace sr;

// Staging area of query_topk_noalloc: the query ids of one call, in a file-scope device array
// so that the call allocates nothing. Every GPU the library runs on holds its own copy, at its
// own address, until the process ends; calls on one GPU share it and see the last call's ids.
// In host code `scratch` is a host-side stand-in, not a device address: host code uses only
// the address hipGetSymbolAddress returns for the device (scratch_ptr below).
constexpr int64_t kScratchIds = 65536;  // 256 KiB per GPU
static __device__ __align__(256) int32_t scratch[kScratchIds];

// Panel columns one column-mode accumulate pass covers by default (see init_impl).
constexpr int kColumnPanelCols = 512;
// Deferred blocks per fused pass at most: the per-pass kernels take one grid row per block.
constexpr int32_t kMaxChunk = 65535;

// Rows longer than kLight entries, kept in sync with the host mirror; the traversal kernels
// process them in chunks (see graph.hip).
struct HeavySet {
  int32_t split = kSplitRows;        // rows with more entries are huge (chunked)
  std::map<int32_t, int8_t> rows;    // listed row -> tier (1 medium, 2 heavy, 3 huge)
  std::map<int32_t, int32_t> cover;  // huge row -> entries its chunks cover
  std::vector<int32_t> med, heavy, huge, hfirst;
  std::vector<int2> chunk;           // (row, first entry) per chunk of the huge rows
  bool dirty = true;
  uint64_t version = 0;              // bumped at every upload (captured graphs depend on it)
  int32_t* d_med = nullptr;
  int32_t* d_heavy = nullptr;
  int32_t* d_huge = nullptr;
  int32_t* d_hfirst = nullptr;
  int2* d_chunk = nullptr;
  double2* d_part = nullptr;   // per-chunk partial sums (traversal scratch)
  uint32_t* d_pflag = nullptr;
  int64_t cap_med = 0, cap_heavy = 0, cap_huge = 0, cap_hfirst = 0, cap_chunk = 0;
};

struct sr_ctx {
  sr_config cfg{};
  hipStream_t stream = nullptr;
  int device = 0;  // the GPU that was current at init (its allocations live there)
  bool poisoned = false;
  bool weighted = false;
  bool updated = false;  // graph changed since init
  int64_t node_cap = 0, edge_cap = 0, slot_cap = 0;
  int64_t p_rows = 0;  // panel rows: node_cap rounded up to 128; rows past n stay zero
  HostGraph g;
  std::vector<int32_t> src0, dst0;  // initial edges (the order of backward's output)
  std::vector<double> w0;
  std::vector<int32_t> slot_edge0;  // in-list slot -> initial edge index

  int32_t* d_adj[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  std::vector<double> Wsum;  // weighted graphs: in-weight sums (the host copy of d_W)
  double* d_in_w = nullptr;
  double* d_out_w = nullptr;
  double* d_W = nullptr;

  SView S{};
  void* S_mem[2] = {nullptr, nullptr};

  // Block store (Example 1.1; cfg.block_store with init_simrank_partitioned): S kept per
  // pair of partition blocks (see BlockStore); the dense S above is then not allocated.
  bool bstore = false;
  int32_t bs_np = 0;
  std::vector<int32_t> bs_n;           // members per block
  std::vector<SView> bs_pairs;         // host copy of the pair table (np x np)
  int32_t *d_bs_part = nullptr, *d_bs_loc = nullptr, *d_bs_mem = nullptr, *d_bs_n = nullptr;
  int64_t* d_bs_off = nullptr;
  SView* d_bs_pairs = nullptr;
  uint32_t* d_bs_flags = nullptr;      // per pass: deferred block x block x {xi, eta}
  int64_t bs_flags_cap = 0;
  BsItem* d_bs_items = nullptr;
  int64_t bs_items_cap = 0;
  int64_t bs_bytes = 0;                // bytes of the pairs' sub-matrices

  double *SI = nullptr, *Sj = nullptr, *QSI = nullptr, *zbuf = nullptr, *Qz = nullptr,
         *zsum = nullptr, *ytmp = nullptr;
  double* P = nullptr;
  double* pairs = nullptr;  // series scratch: two compact (xi_k, eta_k) vectors, node_cap each
  int pld = 0;  // doubles per panel row (one block)
  double* Pb = nullptr;  // fused batch panel: node_cap x (pld * batch_chunk)
  double* wts = nullptr;  // panel-correction weights: 2 * pld * batch_chunk
  uint32_t *suppI = nullptr, *suppJ = nullptr, *Abits = nullptr, *Bbits = nullptr,
           *Ahat = nullptr, *Bhat = nullptr;
  int W = 0;
  int32_t* rowlist = nullptr;
  int32_t* rowlist2 = nullptr;  // rows filled by the transpose copy (launch_aff_mirror)
  int32_t* d_ids = nullptr;  // staging for query ids (capacity ids_cap)
  int64_t ids_cap = 0;
  int64_t* d_cnt = nullptr;
  unsigned long long* d_max = nullptr;
  double* d_sum = nullptr;  // sums over a block's sources of long lists (launch_sum_at)
  int32_t* d_mm = nullptr;  // min / max of caller-supplied device ids (launch_ids_range)
  int32_t* d_blk = nullptr;  // the sources of a batch's long blocks (IdList::dev targets)
  int64_t blk_cap = 0;
  int64_t* h_cnt = nullptr;
  unsigned long long* h_max = nullptr;

  int last_r = 0;          // panel columns of the last unit update (0: none)
  // The last unit update, for its Delta S columns: case (-1 none), its new nodes' ids and
  // diagonals, and for C1 the new sink's column (ylast, its diagonal at j).
  int last_case = -1;
  int32_t last_i = -1, last_j = -1;
  double last_vi = 0.0, last_vj = 0.0;
  double* ylast = nullptr;
  bool last_aff = false;   // AFF bitmaps hold the last update
  std::vector<int32_t> last_plan;

  double* xs = nullptr;    // PartialSim vectors (column mode): (K_ps + 1) pairs x node_cap
  double* xd = nullptr;    // PartialSim: two pair vectors x_t / d (d: row weight of Q)
  // Fused passes: the nodes a pass reaches (bitmap, ascending list, and per pass of a batch
  // the list's length, read on the device by the pass and on the host for statistics).
  uint32_t* d_act_bits = nullptr;
  int32_t* d_act = nullptr;
  int64_t* d_act_cnt = nullptr;
  int64_t act_cnt_cap = 0;
  // Tile skipping (cfg.tile_skip): per pass, the k-steps' tile flags of its blocks, and per
  // low-rank block of a batch and counted k-step the positions of the tiles that skip it.
  uint32_t* d_tflags = nullptr;
  int64_t tflags_cap = 0;
  int32_t* d_skip = nullptr;
  int64_t skip_cap = 0;
  int corr_slots = 0;      // fused batches: slots per chunk at most (2 batch_chunk + 32)
  double* corr = nullptr;  // correction vectors, 2 corr_slots x p_rows
  double* corr_w = nullptr;  // their weights, 2 corr_slots x 64
  int32_t* corr_tab = nullptr;  // slot table of a batch (rstart | sink | rows)
  int64_t corr_tab_cap = 0;

  HeavySet hin, hout;      // heavy in-rows (Q) and out-rows (Q^T)

  int gemm_variant = 0;    // fused GEMM tile variant (launch_lowrank), set by sr_set_tuning
  // Captured K-step series chains of fused batches, one per panel slot of a chunk; a graph
  // holds its panel segment, node count and the in-row tiers' version by value, so it is
  // captured again when any of them changes.
  struct SeriesGraph {
    hipGraphExec_t exec = nullptr;
    const double* P = nullptr;
    int64_t n = -1;
    uint64_t ver = ~0ull;
  };
  std::vector<SeriesGraph> sgraphs;
  hipStream_t cap_stream = nullptr;  // capture only (the context's stream may be the null one)
  int64_t graph_captures = 0, graph_replays = 0;

  bool profiling = false;  // bracket S-update launches with events
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
};

namespace {

sr_status fail_hip(sr_ctx* c) {
  if (c) c->poisoned = true;
  return SR_EHIP;
}

#define HC(expr)                                 \
  do {                                           \
    hipError_t e__ = (expr);                     \
    if (e__ != hipSuccess) return fail_hip(ctx); \
  } while (0)

// The device view of the block store (Example 1.1).
BlockStore bs_view(const sr_ctx* c) {
  BlockStore b{};
  b.pairs = c->d_bs_pairs;
  b.np = c->bs_np;
  b.part = c->d_bs_part;
  b.loc = c->d_bs_loc;
  b.mem = c->d_bs_mem;
  b.mem_off = c->d_bs_off;
  b.mem_n = c->d_bs_n;
  return b;
}

DevQ devq(const sr_ctx* c) {
  DevQ q;
  q.in.start = c->d_adj[0];
  q.in.len = c->d_adj[1];
  q.in.idx = c->d_adj[2];
  q.in.w = c->weighted ? c->d_in_w : nullptr;
  q.W = c->weighted ? c->d_W : nullptr;
  return q;
}

DevAdj devout(const sr_ctx* c) {
  DevAdj a;
  a.start = c->d_adj[3];
  a.len = c->d_adj[4];
  a.idx = c->d_adj[5];
  a.w = c->weighted ? c->d_out_w : nullptr;
  return a;
}

AdjPtrs adjptrs(const sr_ctx* c) {
  AdjPtrs t;
  for (int k = 0; k < 6; ++k) t.p[k] = c->d_adj[k];
  return t;
}

// hipMalloc that leaves no sticky error behind on failure: HIP keeps the last error for
// hipGetLastError, which the kernel launchers read after every launch, so a failed
// allocation would otherwise be reported by the next, unrelated launch.
// Every device allocation of the library goes through dmalloc / dfree, which keep the bytes
// held (all contexts of the process) and their peak for sr_device_bytes.
std::mutex g_mem_mu;
std::unordered_map<void*, size_t> g_mem_live;
int64_t g_mem_now = 0, g_mem_peak = 0;

hipError_t dmalloc(void** p, size_t bytes) {
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return e;
  }
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_mem_live[*p] = bytes;
  g_mem_now += (int64_t)bytes;
  g_mem_peak = std::max(g_mem_peak, g_mem_now);
  return e;
}

hipError_t dfree(void* p) {
  if (!p) return hipSuccess;
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    auto it = g_mem_live.find(p);
    if (it != g_mem_live.end()) {
      g_mem_now -= (int64_t)it->second;
      g_mem_live.erase(it);
    }
  }
  return hipFree(p);
}

template <typename T>
hipError_t dalloc(T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  return dmalloc((void**)p, (size_t)count * sizeof(T));
}

// Records row r's tier after an edit; a change marks the set for upload.
void heavy_touch(HeavySet& H, const SlotList& L, int32_t r) {
  const int32_t len = L.len[r];
  auto it = H.rows.find(r);
  if (len <= kLight) {
    if (it != H.rows.end()) {
      H.rows.erase(it);
      H.cover.erase(r);
      H.dirty = true;
    }
    return;
  }
  const int8_t tier = len > H.split ? 3 : (len > kMedium ? 2 : 1);
  if (it == H.rows.end() || it->second != tier) {
    H.rows[r] = tier;
    H.dirty = true;
  }
  // a huge row's chunks must cover all its entries
  if (tier == 3) {
    auto c = H.cover.find(r);
    if (c == H.cover.end() || len > c->second) H.dirty = true;
  }
}

void heavy_free(HeavySet& H) {
  (void)dfree(H.d_med);
  (void)dfree(H.d_heavy);
  (void)dfree(H.d_huge);
  (void)dfree(H.d_hfirst);
  (void)dfree(H.d_chunk);
  (void)dfree(H.d_part);
  (void)dfree(H.d_pflag);
  H.d_med = H.d_heavy = H.d_huge = H.d_hfirst = nullptr;
  H.d_chunk = nullptr;
  H.d_part = nullptr;
  H.d_pflag = nullptr;
  H.cap_med = H.cap_heavy = H.cap_huge = H.cap_hfirst = H.cap_chunk = 0;
}

template <typename T>
hipError_t upload_list(const std::vector<T>& v, T** d, int64_t* cap) {
  const int64_t cnt = (int64_t)v.size();
  if (cnt > *cap) {
    (void)dfree(*d);
    *d = nullptr;
    const int64_t c = std::max<int64_t>(64, 2 * cnt);
    hipError_t e = dmalloc((void**)d, (size_t)c * sizeof(T));
    if (e != hipSuccess) return e;
    *cap = c;
  }
  if (cnt) return hipMemcpy(*d, v.data(), (size_t)cnt * sizeof(T), hipMemcpyHostToDevice);
  return hipSuccess;
}

// Uploads the medium, heavy and huge lists and the chunk table when they changed. A huge row
// gets len / kChunk + 1 chunks, so it can grow by at least one entry (and up to kChunk)
// before the table must be rebuilt; chunks past the row's current length add nothing.
sr_status heavy_sync(sr_ctx* ctx, HeavySet& H, const SlotList& L) {
  if (!H.dirty) return SR_OK;
  HC(hipStreamSynchronize(ctx->stream));
  H.med.clear();
  H.heavy.clear();
  H.huge.clear();
  H.hfirst.clear();
  H.chunk.clear();
  H.cover.clear();
  for (const auto& rt : H.rows) {
    if (rt.second == 1) {
      H.med.push_back(rt.first);
    } else if (rt.second == 2) {
      H.heavy.push_back(rt.first);
    } else {
      const int32_t nc = L.len[rt.first] / kChunk + 1;
      H.huge.push_back(rt.first);
      H.hfirst.push_back((int32_t)H.chunk.size());
      for (int32_t c = 0; c < nc; ++c) H.chunk.push_back(make_int2(rt.first, c * kChunk));
      H.cover[rt.first] = nc * kChunk;
    }
  }
  H.hfirst.push_back((int32_t)H.chunk.size());
  hipError_t e = upload_list(H.med, &H.d_med, &H.cap_med);
  if (e == hipSuccess) e = upload_list(H.heavy, &H.d_heavy, &H.cap_heavy);
  if (e == hipSuccess) e = upload_list(H.huge, &H.d_huge, &H.cap_huge);
  if (e == hipSuccess) e = upload_list(H.hfirst, &H.d_hfirst, &H.cap_hfirst);
  if (e == hipSuccess) {
    const int64_t old_cap = H.cap_chunk;
    e = upload_list(H.chunk, &H.d_chunk, &H.cap_chunk);
    if (e == hipSuccess && (H.cap_chunk != old_cap || H.d_part == nullptr)) {
      (void)dfree(H.d_part);
      (void)dfree(H.d_pflag);
      H.d_part = nullptr;
      H.d_pflag = nullptr;
      e = dmalloc((void**)&H.d_part, (size_t)std::max<int64_t>(H.cap_chunk, 1) * 16);
      if (e == hipSuccess)
        e = dmalloc((void**)&H.d_pflag, (size_t)std::max<int64_t>(H.cap_chunk, 1) * 4);
    }
  }
  if (e == hipErrorOutOfMemory) return SR_ENOMEM;
  HC(e);
  H.dirty = false;
  ++H.version;
  return SR_OK;
}

HeavyArgs heavy_args(const HeavySet& H) {
  HeavyArgs h;
  h.med = H.d_med;
  h.nmed = (int32_t)H.med.size();
  h.heavy = H.d_heavy;
  h.nheavy = (int32_t)H.heavy.size();
  h.huge = H.d_huge;
  h.nhuge = (int32_t)H.huge.size();
  h.chunk = H.d_chunk;
  h.nchunk = (int32_t)H.chunk.size();
  h.hfirst = H.d_hfirst;
  h.part = H.d_part;
  h.pflag = H.d_pflag;
  return h;
}

sr_status heavy_refresh(sr_ctx* ctx) {
  sr_status r = heavy_sync(ctx, ctx->hin, ctx->g.in);
  if (r == SR_OK) r = heavy_sync(ctx, ctx->hout, ctx->g.out);
  return r;
}

sr_status upload_graph(sr_ctx* ctx) {
  const int64_t nc = ctx->node_cap;
  const SlotList* L[2] = {&ctx->g.in, &ctx->g.out};
  HC(hipStreamSynchronize(ctx->stream));
  for (int l = 0; l < 2; ++l) {
    HC(hipMemcpy(ctx->d_adj[3 * l + 0], L[l]->start.data(), nc * 4, hipMemcpyHostToDevice));
    HC(hipMemcpy(ctx->d_adj[3 * l + 1], L[l]->len.data(), nc * 4, hipMemcpyHostToDevice));
    HC(hipMemcpy(ctx->d_adj[3 * l + 2], L[l]->idx.data(), L[l]->idx.size() * 4,
                 hipMemcpyHostToDevice));
  }
  if (ctx->weighted) {
    HC(hipMemcpy(ctx->d_in_w, ctx->g.in.w.data(), ctx->g.in.w.size() * 8,
                 hipMemcpyHostToDevice));
    HC(hipMemcpy(ctx->d_out_w, ctx->g.out.w.data(), ctx->g.out.w.size() * 8,
                 hipMemcpyHostToDevice));
  }
  return SR_OK;
}

// Whether inserting the edges (i, j) cannot run out of slots in either list (checked by the
// entry points before any launch, so that SR_ECAPACITY leaves the context unchanged).
bool graph_fits(const sr_ctx* ctx, const std::vector<std::pair<int32_t, int32_t>>& ins) {
  std::map<int32_t, int32_t> add_in, add_out;
  for (const auto& ij : ins) {
    add_in[ij.second]++;
    add_out[ij.first]++;
  }
  return ctx->g.in.fits(add_in) && ctx->g.out.fits(add_out);
}

// Applies edge insertions (op > 0) or deletions to the host mirror and the device copy.
// The caller has validated every edge and checked graph_fits for the insertions.
// Weighted graphs: the in-weight sum of sink j from its row of the mirror, in slot order.
double row_weight(const sr_ctx* ctx, int32_t j) {
  const SlotList& L = ctx->g.in;
  double w = 0.0;
  for (int32_t p = 0; p < L.len[j]; ++p) w += L.w[L.start[j] + p];
  return w;
}

WPtrs wptrs(const sr_ctx* c) {
  WPtrs t;
  t.p[0] = c->d_in_w;
  t.p[1] = c->d_out_w;
  t.p[2] = c->d_W;
  return t;
}

// Launches the weight writes (array, index, value) in patches.
sr_status patch_weights(sr_ctx* ctx, const std::vector<std::pair<std::pair<int32_t, int32_t>,
                                                                double>>& wr) {
  WPatch p;
  p.count = 0;
  for (const auto& x : wr) {
    p.array[p.count] = x.first.first;
    p.index[p.count] = x.first.second;
    p.value[p.count] = x.second;
    if (++p.count == WPatch::MAX) {
      HC(launch_patch_w(wptrs(ctx), p, ctx->stream));
      p.count = 0;
    }
  }
  if (p.count) HC(launch_patch_w(wptrs(ctx), p, ctx->stream));
  return SR_OK;
}

// Weighted graphs: sets the weight of the existing edge i -> j to w (mirror and device: the
// two slot weights and W[j]).
sr_status reweight_edge(sr_ctx* ctx, int32_t i, int32_t j, double w) {
  SlotList& in = ctx->g.in;
  SlotList& out = ctx->g.out;
  const int32_t pi = in.find(j, i), po = out.find(i, j);
  if (pi < 0 || po < 0) return SR_ENOENT;
  in.w[in.start[j] + pi] = w;
  out.w[out.start[i] + po] = w;
  ctx->Wsum[j] = row_weight(ctx, j);
  ctx->updated = true;
  return patch_weights(ctx, {{{0, in.start[j] + pi}, w},
                             {{1, out.start[i] + po}, w},
                             {{2, j}, ctx->Wsum[j]}});
}

sr_status edit_graph(sr_ctx* ctx, const std::vector<std::pair<int32_t, int32_t>>& e, int op,
                     const std::vector<double>* wts = nullptr) {
  std::vector<Write> wi, wo;
  std::vector<int32_t> mi, mo;
  bool full = false, cap_err = false;
  for (size_t k = 0; k < e.size(); ++k) {
    const int32_t i = e[k].first, j = e[k].second;
    if (op > 0) {
      const double wt = wts ? (*wts)[k] : 1.0;
      const int r1 = ctx->g.in.insert(j, i, wt, wi, mi);
      const int r2 = ctx->g.out.insert(i, j, wt, wo, mo);
      full |= (r1 >= 2) || (r2 >= 2);
      cap_err |= (r1 == 3) || (r2 == 3);
      ctx->g.edges.insert(HostGraph::key(i, j));
      ctx->g.m++;
    } else {
      ctx->g.in.remove(j, i, wi);
      ctx->g.out.remove(i, j, wo);
      ctx->g.edges.erase(HostGraph::key(i, j));
      ctx->g.m--;
    }
    heavy_touch(ctx->hin, ctx->g.in, j);
    heavy_touch(ctx->hout, ctx->g.out, i);
  }
  ctx->updated = true;
  std::vector<std::pair<std::pair<int32_t, int32_t>, double>> wr;  // weight writes
  if (ctx->weighted) {
    std::set<int32_t> sinks;
    for (auto& ij : e) sinks.insert(ij.second);
    for (int32_t j : sinks) {
      ctx->Wsum[j] = row_weight(ctx, j);
      wr.push_back({{2, j}, ctx->Wsum[j]});
    }
  }
  {
    sr_status hs = heavy_refresh(ctx);
    if (hs != SR_OK) {
      // the mirror has changed: a failure here cannot leave the context as it was
      ctx->poisoned = true;
      return hs;
    }
  }
  if (cap_err) {
    // not reachable after graph_fits; the mirror no longer matches the edges it lists
    ctx->poisoned = true;
    return SR_EHIP;
  }
  if (full) {
    sr_status us = upload_graph(ctx);
    if (us == SR_OK && ctx->weighted)
      HC(hipMemcpy(ctx->d_W, ctx->Wsum.data(), ctx->Wsum.size() * 8, hipMemcpyHostToDevice));
    return us;
  }
  // Moved rows: upload their slots; then patch every touched (array, index) with the mirror's
  // final value (unique addresses per launch, so the writes of one launch commute).
  const SlotList* L[2] = {&ctx->g.in, &ctx->g.out};
  std::vector<int32_t>* M[2] = {&mi, &mo};
  std::vector<Write>* Wv[2] = {&wi, &wo};
  bool synced = false;
  for (int l = 0; l < 2; ++l) {
    for (int32_t r : *M[l]) {
      if (!synced) {
        HC(hipStreamSynchronize(ctx->stream));
        synced = true;
      }
      const int32_t st = L[l]->start[r], ln = L[l]->len[r];
      HC(hipMemcpy(ctx->d_adj[3 * l + 2] + st, L[l]->idx.data() + st, (size_t)ln * 4,
                   hipMemcpyHostToDevice));
      if (ctx->weighted)
        HC(hipMemcpy((l == 0 ? ctx->d_in_w : ctx->d_out_w) + st, L[l]->w.data() + st,
                     (size_t)ln * 8, hipMemcpyHostToDevice));
      Wv[l]->push_back({0, r, 0});
      Wv[l]->push_back({1, r, 0});
    }
  }
  std::set<std::pair<int32_t, int32_t>> touched;
  for (int l = 0; l < 2; ++l)
    for (auto& w : *Wv[l]) touched.insert({3 * l + w.array, w.index});
  Patch p;
  p.count = 0;
  for (auto& t : touched) {
    const int l = t.first / 3, a = t.first % 3;
    const std::vector<int32_t>& src =
        a == 0 ? L[l]->start : (a == 1 ? L[l]->len : L[l]->idx);
    p.array[p.count] = t.first;
    p.index[p.count] = t.second;
    p.value[p.count] = src[t.second];
    if (++p.count == Patch::MAX) {
      HC(launch_patch(adjptrs(ctx), p, ctx->stream));
      p.count = 0;
    }
  }
  if (p.count) HC(launch_patch(adjptrs(ctx), p, ctx->stream));
  if (ctx->weighted) {
    // the weight of every slot whose index was written moves with it
    for (auto& t : touched)
      if (t.first % 3 == 2) wr.push_back({{t.first / 3, t.second}, L[t.first / 3]->w[t.second]});
    return patch_weights(ctx, wr);
  }
  return SR_OK;
}

// Runs one launch of a call's dominant kernel, bracketed by events on the context stream
// when profiling is on.
template <typename F>
hipError_t profiled(sr_ctx* ctx, F&& launch) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->profiling) {
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
    if (e != hipSuccess) return e;
  }
  hipError_t e = launch();
  if (e == hipSuccess && ctx->profiling) {
    e = hipEventRecord(e1, ctx->stream);
    ctx->prof_events.push_back({e0, e1});
  }
  return e;
}

// Launches the S update (or the column output), profiled.
hipError_t run_lowrank(sr_ctx* ctx, const LowRankArgs& la) {
  return profiled(ctx, [&]() { return launch_lowrank(la, ctx->stream); });
}

// Ids v[off .. off + cnt) as a kernel list: by value up to IdList::MAX, otherwise the device
// copy at dev (which the caller has uploaded; a long list without one is a caller error).
IdList idlist(const std::vector<int32_t>& v, size_t off, size_t cnt,
              const int32_t* dev = nullptr) {
  IdList l;
  l.count = (int32_t)cnt;
  if (cnt > (size_t)IdList::MAX) {
    l.dev = dev;
  } else {
    for (size_t t = 0; t < cnt; ++t) l.id[t] = v[off + t];
  }
  return l;
}

// Uploads the source lists longer than IdList::MAX of a batch's blocks, back to back, to
// ctx->d_blk; dev_of[b] receives block b's device list (null for short lists).
template <typename BlockT>
sr_status stage_long_lists(sr_ctx* ctx, const std::vector<BlockT>& plan,
                           std::vector<const int32_t*>& dev_of) {
  dev_of.assign(plan.size(), nullptr);
  std::vector<int32_t> ids;
  std::vector<int64_t> off(plan.size(), -1);
  for (size_t b = 0; b < plan.size(); ++b) {
    if (plan[b].I.size() <= (size_t)IdList::MAX) continue;
    off[b] = (int64_t)ids.size();
    ids.insert(ids.end(), plan[b].I.begin(), plan[b].I.end());
  }
  if (ids.empty()) return SR_OK;
  // earlier work may still read the previous lists
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return fail_hip(ctx);
  if ((int64_t)ids.size() > ctx->blk_cap) {
    (void)dfree(ctx->d_blk);
    ctx->d_blk = nullptr;
    ctx->blk_cap = 0;
    const int64_t c = std::max<int64_t>(4096, 2 * (int64_t)ids.size());
    if (dmalloc((void**)&ctx->d_blk, (size_t)c * 4) != hipSuccess) return SR_ENOMEM;
    ctx->blk_cap = c;
  }
  if (hipMemcpy(ctx->d_blk, ids.data(), ids.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return fail_hip(ctx);
  for (size_t b = 0; b < plan.size(); ++b)
    if (off[b] >= 0) dev_of[b] = ctx->d_blk + off[b];
  return SR_OK;
}

AffArgs aff_args(const sr_ctx* c, int64_t n) {
  AffArgs a;
  a.n = n;
  a.W = c->W;
  a.K = c->cfg.K;
  a.A = c->Abits;
  a.B = c->Bbits;
  return a;
}

// Deferred application inside a fused batch: the batch panel holds one n x pld panel per
// deferred block, gstride doubles apart (block-major, so that the series traversal of a block
// gathers from rows of pld doubles). A block writes its (xi_k, eta_k) pairs into panel
// r_prev / pld, and S_t columns are corrected by the r_prev deferred columns before gamma.
// With incremental corrections, cI / cJ are the block's correction vectors (added to the
// gathered columns) and the deferred panel is not read.
struct FusedTarget {
  double* P;
  int64_t gstride;
  int pld;
  int r_prev;
  bool incremental = false;
  const double* cI = nullptr;
  const double* cJ = nullptr;
};

// The K steps of eq (16a) of a deferred block that writes the panel segment P, replayed from
// the captured graph of its chunk slot (captured on a private stream, launched on the
// context's stream, so it runs in order with the block's other launches).
sr_status series_replay(sr_ctx* ctx, int slot, double* P, int64_t n_work) {
  if ((int)ctx->sgraphs.size() <= slot) ctx->sgraphs.resize(slot + 1);
  sr_ctx::SeriesGraph& sg = ctx->sgraphs[slot];
  const uint64_t ver = ctx->hin.version;
  if (!sg.exec || sg.P != P || sg.n != n_work || sg.ver != ver) {
    if (sg.exec) {
      (void)hipGraphExecDestroy(sg.exec);
      sg.exec = nullptr;
    }
    if (!ctx->cap_stream) HC(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HC(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    const DevQ q = devq(ctx);
    const HeavyArgs h = heavy_args(ctx->hin);
    hipError_t e = hipSuccess;
    for (int k = 0; k < ctx->cfg.K && e == hipSuccess; ++k)
      e = launch_series_step(q, h, n_work, P, ctx->pld, k, ctx->cfg.C, 1.0, nullptr,
                             ctx->cap_stream, ctx->pairs, ctx->node_cap);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (e == hipSuccess) e = ee;
    if (e == hipSuccess) e = hipGraphInstantiate(&sg.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) sg.exec = nullptr;
    HC(e);
    sg.P = P;
    sg.n = n_work;
    sg.ver = ver;
    ++ctx->graph_captures;
  }
  HC(hipGraphLaunch(sg.exec, ctx->stream));
  ++ctx->graph_replays;
  return SR_OK;
}

// One low-rank block (Table 2 rows C0 insert/delete, or C2): gamma from the old S and graph,
// affected areas, graph edit, K series steps on the new graph, and the S update.
//   case_id 0: sources I exist; case_id 2: sources I are new nodes (isolated until now).
//   n_work: node count the kernels cover (includes new and not yet created nodes).
//   Weighted graphs (one source): alpha != 0 is the scale a of Delta Q = e_j a (e_i -
//   Q[j, :])^T (case 0: gamma kind 3; case 2: a = w / (W_j + w)); reweight: the edge exists
//   and only its weight becomes wt, otherwise insertions carry the weight wt.
sr_status lowrank_block(sr_ctx* ctx, int case_id, int op, const std::vector<int32_t>& I,
                        int32_t j, int64_t n_work, sr_update_stats* st,
                        const FusedTarget* ft = nullptr, const int32_t* I_dev = nullptr,
                        double alpha = 0.0, bool reweight = false, double wt = 1.0) {
  const double C = ctx->cfg.C;
  const int K = ctx->cfg.K;
  const int delta = (int)I.size();
  const int64_t dj = ctx->g.in.len[j];
  const bool prune = ctx->cfg.prune != 0 && ft == nullptr;
  double* P = ft ? ft->P + (int64_t)(ft->r_prev / ft->pld) * ft->gstride : ctx->P;
  const int pld = ctx->pld;
  const bool direct = (case_id == 0) && ctx->cfg.gamma_form == SR_GAMMA_DIRECT &&
                      !ctx->weighted && alpha == 0.0;
  hipStream_t s = ctx->stream;
  const DevQ q = devq(ctx);

  GammaArgs ga{};
  ga.kind = case_id == 2 ? 2 : (alpha != 0.0 ? 3 : (direct ? 1 : 0));
  ga.alpha = alpha;
  ga.op = op;
  ga.j = j;
  ga.delta = delta;
  ga.dj = dj;
  ga.C = C;
  ga.xi0 = case_id == 2 ? (alpha > 0.0 ? C * alpha : C * (double)delta / (double)(dj + delta))
                       : C;
  ga.I = idlist(I, 0, case_id == 0 ? I.size() : 0, I_dev);

  // S[:, I] (with supports) and S[:, j] from the old S.
  const IdList src_rows = ga.I;
  if (ctx->bstore)
    HC(launch_bs_gather_rows(bs_view(ctx), n_work, src_rows, j, ctx->SI, ctx->Sj,
                             ft ? ft->cI : nullptr, ft ? ft->cJ : nullptr, s));
  else
    HC(launch_gather_rows(ctx->S, n_work, src_rows, 0, j, ctx->SI, ctx->Sj, ctx->suppI,
                          ctx->suppJ, s, ft ? ft->cI : nullptr, ft ? ft->cJ : nullptr));
  if (ft && !ft->incremental && ft->r_prev > 0)
    HC(launch_panel_correct(ft->P, ft->pld, ft->gstride, ft->r_prev, n_work, src_rows, j, ctx->wts,
                            ctx->SI, ctx->Sj, s));
  const AffArgs aa = aff_args(ctx, n_work);
  const int64_t W = ctx->W;
  uint32_t* A = ctx->Abits;
  uint32_t* B = ctx->Bbits;
  if (prune) {
    HC(hipMemsetAsync(A, 0, (size_t)(K + 1) * W * 4, s));
    HC(hipMemsetAsync(B, 0, (size_t)(K + 1) * W * 4, s));
  }
  const HeavyArgs hin = heavy_args(ctx->hin);
  if (case_id == 0) {
    // Q_old S[:, I]; in the same traversal F1 = out_old(supp S[I, :]) goes into B_0.
    HC(launch_spmv_q(q, hin, n_work, ctx->SI, ctx->QSI, 1.0, s, nullptr, 1.0,
                     prune ? ctx->suppI : nullptr, prune ? B : nullptr, W));
    if (direct) {
      if (dj > 0) HC(launch_gather_inrows(ctx->S, n_work, q, j, ctx->zsum, s));
      HC(launch_direct_z(ga, n_work, ctx->SI, ctx->zsum, ctx->zbuf, s));
      HC(launch_spmv_q(q, hin, n_work, ctx->zbuf, ctx->Qz, 1.0, s));
    }
    if (ga.I.dev) {
      // a long list: the sum over I (of S[:, I], or of z) once, not per thread
      HC(launch_sum_at(direct ? ctx->zbuf : ctx->SI, ga.I, ctx->d_sum, s));
      ga.sumI = ctx->d_sum;
    }
  }
  if (st) HC(hipMemsetAsync(ctx->d_max, 0, sizeof(unsigned long long), s));
  HC(launch_gamma(ga, n_work, ctx->SI, ctx->Sj, ctx->QSI, ctx->zbuf, ctx->Qz, P, pld,
                  st ? ctx->d_max : nullptr, s));
  if (prune) {
    // F2 = supp S[j, :] unless row j of Q is empty before an insertion / after a deletion
    // (case C2: B_0 = supp S[j, :] | {j}).
    const int f2 = case_id == 2 ? 1 : (op > 0 ? (dj > 0) : (dj > delta));
    HC(launch_aff_level0(aa, ctx->suppJ, f2, j, s));
  }

  // Graph edit.
  std::vector<std::pair<int32_t, int32_t>> edges;
  for (int32_t i : I) edges.push_back({i, j});
  const std::vector<double> wts(I.size(), wt);
  sr_status es = reweight ? reweight_edge(ctx, I[0], j, wt) : edit_graph(ctx, edges, op, &wts);
  if (es != SR_OK) return es;
  const DevQ q_new = devq(ctx);
  const HeavyArgs hin_new = heavy_args(ctx->hin);

  // K steps of eq (16a) on the new graph; level k+1 of the affected areas in the same pass:
  // A_{k+1} = out_new(A_0 | A_k), B_{k+1} = out_new(B_0 | B_k). A deferred block of a fused
  // batch (no affected areas) replays its chain from a captured graph.
  if (ft && !prune && ctx->cfg.graphs && K > 0)
    return series_replay(ctx, ft->r_prev / ft->pld, P, n_work);
  for (int k = 0; k < K; ++k) {
    AffLevel al;
    al.a0 = A;
    al.a1 = k >= 1 ? A + (int64_t)k * W : nullptr;
    al.aout = A + (int64_t)(k + 1) * W;
    al.b0 = B;
    al.b1 = k >= 1 ? B + (int64_t)k * W : nullptr;
    al.bout = B + (int64_t)(k + 1) * W;
    al.nwords = W;
    HC(launch_series_step(q_new, hin_new, n_work, P, pld, k, C, 1.0, prune ? &al : nullptr,
                          s, ctx->pairs, ctx->node_cap));
  }
  if (ft) return SR_OK;  // applied later by the batch's fused pass
  if (prune)
    HC(launch_aff_compact(aa, ctx->Ahat, ctx->Bhat, ctx->rowlist, ctx->rowlist2, ctx->d_cnt, s));

  LowRankArgs la{};
  la.S = ctx->S;
  la.P = ctx->P;
  la.pld = ctx->pld;
  la.gstride = ctx->p_rows * ctx->pld;
  la.p_rows = ctx->p_rows;
  la.r = 2 * (K + 1);
  la.ncols = n_work;
  if (prune) {
    la.rows = ctx->rowlist;
    la.nrows_dev = ctx->d_cnt + 3;
    la.nrows = n_work;
    la.Ahat = ctx->Ahat;
    la.Bhat = ctx->Bhat;
  } else {
    la.rows = nullptr;
    la.nrows = n_work;
    // above 32 columns the GEMM form runs over whole 32-column chunks; the panel's columns
    // past 2 (K + 1) are zero
    if (la.r > 32) la.r = ctx->pld;
  }
  HC(run_lowrank(ctx, la));
  if (prune) HC(launch_aff_mirror(ctx->S, ctx->rowlist, ctx->rowlist2, ctx->d_cnt, s));
  ctx->last_r = 2 * (K + 1);
  ctx->last_aff = prune;

  if (st) {
    if (prune) HC(hipMemcpyAsync(ctx->h_cnt, ctx->d_cnt, 4 * sizeof(int64_t),
                                 hipMemcpyDeviceToHost, s));
    HC(hipMemcpyAsync(ctx->h_max, ctx->d_max, sizeof(unsigned long long),
                      hipMemcpyDeviceToHost, s));
    HC(hipStreamSynchronize(s));
    double gmax;
    memcpy(&gmax, ctx->h_max, sizeof(double));
    st->case_id = case_id;
    st->op = op;
    st->d_j = dj;
    if (prune) {
      st->aff_A = ctx->h_cnt[0];
      st->aff_B = ctx->h_cnt[1];
      st->aff_AB = ctx->h_cnt[2];
      st->pairs = 2 * ctx->h_cnt[0] * ctx->h_cnt[1] - ctx->h_cnt[2] * ctx->h_cnt[2];
    } else {
      st->aff_A = st->aff_B = st->aff_AB = n_work;
      st->pairs = n_work * n_work;
    }
    st->bound = 2.0 * ga.xi0 * pow(C, K + 1) / (1.0 - C) * gmax;
  }
  return SR_OK;
}

// C1 block (Theorem 8, Table 2 row C1): existing sources I, new sink j.
sr_status c1_block(sr_ctx* ctx, const std::vector<int32_t>& I, int32_t j, int64_t n_work,
                   const FusedTarget* ft = nullptr, const int32_t* I_dev = nullptr,
                   double wt = 1.0) {
  hipStream_t s = ctx->stream;
  const double C = ctx->cfg.C;
  const IdList il = idlist(I, 0, I.size(), I_dev);
  HC(launch_gather_rows(ctx->S, n_work, il, 0, -1, ctx->SI, nullptr, ctx->suppI, nullptr, s,
                        ft ? ft->cI : nullptr, nullptr));
  if (ft && !ft->incremental && ft->r_prev > 0)
    HC(launch_panel_correct(ft->P, ft->pld, ft->gstride, ft->r_prev, n_work, il, -1, ctx->wts, ctx->SI,
                            nullptr, s));
  // y = (C / delta) Q S[:, I] and the corner into ylast (kept as the update's Delta S column)
  HC(launch_spmv_q(devq(ctx), heavy_args(ctx->hin), n_work, ctx->SI, ctx->ylast,
                   C / (double)I.size(), s));
  if (il.dev) HC(launch_sum_at(ctx->SI, il, ctx->d_sum, s));
  HC(launch_c1_corner(ctx->ylast, j, ctx->SI, il, C, s, il.dev ? ctx->d_sum : nullptr));
  HC(launch_c1_border(ctx->S, n_work, j, ctx->ylast, ctx->SI, il, C, s,
                      il.dev ? ctx->d_sum : nullptr));
  std::vector<std::pair<int32_t, int32_t>> e;
  for (int32_t i : I) e.push_back({i, j});
  const std::vector<double> wts(I.size(), wt);
  return edit_graph(ctx, e, +1, &wts);
}

sr_status set_diags(sr_ctx* ctx, const std::vector<std::pair<int32_t, double>>& d) {
  DiagList dl;
  dl.count = 0;
  for (auto& x : d) {
    dl.id[dl.count] = x.first;
    dl.val[dl.count] = x.second;
    if (++dl.count == DiagList::MAX) {
      HC(launch_set_diag(ctx->S, dl, ctx->stream));
      dl.count = 0;
    }
  }
  if (dl.count) HC(launch_set_diag(ctx->S, dl, ctx->stream));
  return SR_OK;
}

// C3 block (Algorithm 5, Table 2 row C3): new sources I and new sink j.
sr_status c3_block(sr_ctx* ctx, const std::vector<int32_t>& I, int32_t j, double wt = 1.0) {
  const double C = ctx->cfg.C;
  std::vector<std::pair<int32_t, double>> d;
  for (int32_t i : I) d.push_back({i, 1.0 - C});
  d.push_back({j, (1.0 - C) * (1.0 + C / (double)I.size())});
  sr_status r = set_diags(ctx, d);
  if (r != SR_OK) return r;
  std::vector<std::pair<int32_t, int32_t>> e;
  for (int32_t i : I) e.push_back({i, j});
  const std::vector<double> wts(I.size(), wt);
  return edit_graph(ctx, e, +1, &wts);
}

// PartialSim (section 7): column q of the K_ps-term SimRank into out (n values).
// x_0 = e_q, x_t = Q^T x_{t-1} (t = 1..K); y = x_K, y <- x_{K-t} + C Q y (t = 1..K); (1 - C) y.
// The Q^T products read x_{t-1} divided by the row weights of Q (two alternating buffers).
// With several ids the start is their indicator, and by linearity the result is the sum of
// their columns (S[:, I] of Table 2).
sr_status partial_sim(sr_ctx* ctx, const IdList& ids, double* out) {
  const int64_t n = ctx->g.n;
  const int Kp = ctx->cfg.K_ps > 0 ? ctx->cfg.K_ps : ctx->cfg.K;
  const double C = ctx->cfg.C;
  hipStream_t s = ctx->stream;
  const DevQ dq = devq(ctx);
  const DevAdj out_l = devout(ctx);
  auto x = [&](int t) { return ctx->xs + (int64_t)t * ctx->node_cap; };
  auto xd = [&](int t) { return ctx->xd + (int64_t)(t & 1) * ctx->node_cap; };
  HC(launch_indicator(x(0), n, ids, s, &dq, xd(0)));
  const HeavyArgs hin = heavy_args(ctx->hin), hout = heavy_args(ctx->hout);
  for (int t = 1; t <= Kp; ++t)
    HC(launch_spmv_qt(dq, out_l, hout, n, xd(t - 1), x(t), t < Kp ? xd(t) : nullptr, 1.0, s));
  const double* y = x(Kp);
  for (int t = 1; t <= Kp; ++t) {
    double* dst = (t == Kp) ? out : ((t & 1) ? ctx->ytmp : ctx->zbuf);
    HC(launch_spmv_q(dq, hin, n, y, dst, C, s, x(Kp - t), t == Kp ? (1.0 - C) : 1.0));
    y = dst;
  }
  if (Kp == 0) HC(hipMemcpyAsync(out, x(0), (size_t)n * 8, hipMemcpyDeviceToDevice, s));
  return SR_OK;
}

// Two PartialSim columns at once, S[:, a] into outa and S[:, b] into outb, as pairs of vectors
// (the recurrences are the same linear maps, so each product reads both in one gather). The
// Horner pass writes y_t over x_{K-t}, the base it adds, row by row.
sr_status partial_sim2(sr_ctx* ctx, const IdList& a, const IdList& b, double* outa,
                       double* outb) {
  const int64_t n = ctx->g.n;
  const int Kp = ctx->cfg.K_ps > 0 ? ctx->cfg.K_ps : ctx->cfg.K;
  if (Kp == 0) {
    sr_status r = partial_sim(ctx, a, outa);
    return r == SR_OK ? partial_sim(ctx, b, outb) : r;
  }
  const double C = ctx->cfg.C;
  hipStream_t s = ctx->stream;
  const DevQ dq = devq(ctx);
  const DevAdj out_l = devout(ctx);
  auto x2 = [&](int t) { return ctx->xs + (int64_t)t * 2 * ctx->node_cap; };
  auto xd2 = [&](int t) { return ctx->xd + (int64_t)(t & 1) * 2 * ctx->node_cap; };
  HC(launch_indicator2(x2(0), n, a, b, s, dq, xd2(0)));
  const HeavyArgs hin = heavy_args(ctx->hin), hout = heavy_args(ctx->hout);
  for (int t = 1; t <= Kp; ++t)
    HC(launch_spmv_qt2(dq, out_l, hout, n, xd2(t - 1), x2(t), t < Kp ? xd2(t) : nullptr, 1.0,
                       s));
  for (int t = 1; t <= Kp; ++t) {
    double* base = x2(Kp - t);
    if (t == Kp)
      HC(launch_spmv_q2(dq, hin, n, x2(Kp - t + 1), nullptr, C, s, base, 1.0 - C, outa, outb));
    else
      HC(launch_spmv_q2(dq, hin, n, x2(Kp - t + 1), base, C, s, base, 1.0));
  }
  return SR_OK;
}

bool valid_ctx(sr_ctx* c) { return c != nullptr; }

// The current edges in sink-major slot order: slot -> position (the order sr_edges reports
// after an update), -1 for unused slots.
std::vector<int32_t> slot_edges(const sr_ctx* ctx) {
  const SlotList& L = ctx->g.in;
  std::vector<int32_t> se(L.idx.size(), -1);
  int32_t k = 0;
  for (int64_t j = 0; j < ctx->g.n; ++j)
    for (int32_t p = 0; p < L.len[j]; ++p) se[L.start[j] + p] = k++;
  return se;
}

// Device addresses of `scratch`, one per GPU, resolved once per device at context creation
// (with that device current) and kept for the life of the process.
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
int32_t* scratch_ptr[kMaxDevices] = {};

sr_status resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return SR_EINVAL;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_ptr[dev]) return SR_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    return SR_EHIP;
  }
  scratch_ptr[dev] = static_cast<int32_t*>(p);
  return SR_OK;
}

// Checks that every id of the device pair arrays lies in [0, n) before they are used as
// addresses (synchronises the stream): SR_ERANGE otherwise.
sr_status check_pair_ids(sr_ctx* ctx, int64_t np, const int32_t* a, const int32_t* b) {
  if (np <= 0) return SR_OK;
  HC(launch_ids_range(a, b, np, ctx->d_mm, ctx->stream));
  HC(hipMemcpyAsync(ctx->h_cnt + 6, ctx->d_mm, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                    ctx->stream));
  HC(hipStreamSynchronize(ctx->stream));
  int32_t mm[2];
  memcpy(mm, ctx->h_cnt + 6, sizeof(mm));
  return (mm[0] < 0 || (int64_t)mm[1] >= ctx->g.n) ? SR_ERANGE : SR_OK;
}

}  // namespace

extern "C" {

const char* sr_strerror(sr_status s) {
  switch (s) {
    case SR_OK: return "ok";
    case SR_EINVAL: return "invalid argument";
    case SR_ERANGE: return "node id out of range or new node ids not dense";
    case SR_EEXIST: return "edge exists";
    case SR_ENOENT: return "edge does not exist";
    case SR_ESELF: return "self-loop";
    case SR_ECAPACITY: return "capacity exceeded";
    case SR_ENOMEM: return "out of memory";
    case SR_EMODE: return "not available in this mode";
    case SR_EHIP: return "HIP runtime error (context poisoned)";
  }
  return "unknown status";
}

sr_status sr_default_config(sr_config* cfg) {
  if (!cfg) return SR_EINVAL;
  memset(cfg, 0, sizeof(*cfg));
  cfg->C = 0.6;
  cfg->K = 15;
  cfg->K_ps = 30;
  cfg->s_prec = SR_S_FP64;
  cfg->mode = SR_DENSE;
  cfg->gamma_form = SR_GAMMA_CLOSED;
  cfg->prune = 1;
  cfg->node_cap = 0;
  cfg->edge_cap = 0;
  cfg->init_tol = 1e-15;
  cfg->init_max_iter = 400;
  cfg->batch_chunk = 0;  // mode default, resolved by init_simrank
  cfg->fused_batch = 1;
  cfg->split_rows = kSplitRows;
  cfg->graphs = 1;
  cfg->tile_skip = 1;
  return SR_OK;
}

sr_status sr_destroy(sr_ctx* ctx) {
  if (!ctx) return SR_OK;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& g : ctx->sgraphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (auto& ev : ctx->prof_events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  for (int k = 0; k < 6; ++k) (void)dfree(ctx->d_adj[k]);
  (void)dfree(ctx->d_in_w);
  (void)dfree(ctx->d_out_w);
  (void)dfree(ctx->d_W);
  (void)dfree(ctx->S_mem[0]);
  (void)dfree(ctx->S_mem[1]);
  for (SView& v : ctx->bs_pairs) (void)dfree(v.d);
  int32_t* bsi[] = {ctx->d_bs_part, ctx->d_bs_loc, ctx->d_bs_mem, ctx->d_bs_n};
  for (int32_t* p : bsi) (void)dfree(p);
  (void)dfree(ctx->d_bs_off);
  (void)dfree(ctx->d_bs_pairs);
  (void)dfree(ctx->d_bs_flags);
  (void)dfree(ctx->d_bs_items);
  (void)dfree(ctx->d_act_bits);
  (void)dfree(ctx->d_act);
  (void)dfree(ctx->d_act_cnt);
  (void)dfree(ctx->d_tflags);
  (void)dfree(ctx->d_skip);
  double* dd[] = {ctx->SI, ctx->Sj, ctx->QSI, ctx->zbuf, ctx->Qz, ctx->zsum, ctx->ytmp, ctx->ylast,
                  ctx->P, ctx->pairs, ctx->Pb, ctx->wts, ctx->xs, ctx->xd, ctx->corr,
                  ctx->corr_w};
  for (double* p : dd) (void)dfree(p);
  uint32_t* bb[] = {ctx->suppI, ctx->suppJ, ctx->Abits, ctx->Bbits, ctx->Ahat, ctx->Bhat};
  for (uint32_t* p : bb) (void)dfree(p);
  (void)dfree(ctx->rowlist);
  (void)dfree(ctx->rowlist2);
  (void)dfree(ctx->d_ids);
  (void)dfree(ctx->corr_tab);
  heavy_free(ctx->hin);
  heavy_free(ctx->hout);
  (void)dfree(ctx->d_cnt);
  (void)dfree(ctx->d_max);
  (void)dfree(ctx->d_sum);
  (void)dfree(ctx->d_mm);
  (void)dfree(ctx->d_blk);
  (void)hipHostFree(ctx->h_cnt);
  (void)hipHostFree(ctx->h_max);
  delete ctx;
  return SR_OK;
}

static sr_status init_impl(sr_ctx** out, int64_t n, int64_t m, const int32_t* src,
                           const int32_t* dst, const double* weight, const sr_config* cfg_in,
                           const void* S0, void* hip_stream, const int32_t* tree_parent,
                           const int32_t* tree_depth, const int32_t* block_part);

namespace {

// Block store (Example 1.1): pair allocation, initialisation and the fused pass.
constexpr int32_t kMaxStoreBlocks = 4096;  // the pair table holds np^2 views
constexpr int64_t kStoreTopkRows = 256;    // query rows staged at a time for top-k

// Copies host ids into ctx->d_ids (grown as needed) once earlier work has read it.
sr_status stage_ids(sr_ctx* ctx, const int32_t* ids, int64_t cnt) {
  HC(hipStreamSynchronize(ctx->stream));
  if (ctx->ids_cap < cnt) {
    (void)dfree(ctx->d_ids);
    ctx->d_ids = nullptr;
    ctx->ids_cap = 0;
    if (dalloc(&ctx->d_ids, cnt) != hipSuccess) return SR_ENOMEM;
    ctx->ids_cap = cnt;
  }
  HC(hipMemcpy(ctx->d_ids, ids, (size_t)cnt * 4, hipMemcpyHostToDevice));
  return SR_OK;
}

// Pair (p, q), p <= q: a zero-filled mem_n[p] x mem_n[q] sub-matrix in the store's precision.
// The caller uploads the pair table afterwards.
sr_status bs_alloc_pair(sr_ctx* ctx, int32_t p, int32_t q) {
  SView& v = ctx->bs_pairs[(int64_t)p * ctx->bs_np + q];
  if (v.d) return SR_OK;
  const size_t es = ctx->cfg.s_prec == SR_S_FP32 ? 4 : 8;
  const size_t bytes = (size_t)ctx->bs_n[p] * (size_t)ctx->bs_n[q] * es;
  void* mem = nullptr;
  if (dmalloc(&mem, bytes) != hipSuccess) return SR_ENOMEM;
  v.prec = ctx->cfg.s_prec;
  v.ld = ctx->bs_n[q];
  v.d = (double*)mem;
  v.hl = (float2*)mem;
  v.hi = (float*)mem;
  ctx->bs_bytes += (int64_t)bytes;
  HC(hipMemsetAsync(mem, 0, bytes, ctx->stream));
  return SR_OK;
}

sr_status bs_upload_pairs(sr_ctx* ctx) {
  HC(hipStreamSynchronize(ctx->stream));  // earlier kernels read the old table
  HC(hipMemcpy(ctx->d_bs_pairs, ctx->bs_pairs.data(), ctx->bs_pairs.size() * sizeof(SView),
               hipMemcpyHostToDevice));
  return SR_OK;
}

// S of the blocks' own edges into the diagonal pairs, block by block: each block's fixed
// point on a context of its own nodes (float64), converted into the store's precision.
sr_status block_store_init(sr_ctx* ctx, int64_t n, int64_t m, const int32_t* src,
                           const int32_t* dst, const int32_t* part, void* hip_stream) {
  int32_t np = 0;
  for (int64_t v = 0; v < n; ++v) np = std::max(np, part[v] + 1);
  if (np > kMaxStoreBlocks) return SR_ECAPACITY;
  ctx->bstore = true;
  ctx->bs_np = np;
  std::vector<std::vector<int32_t>> mem(np), bs(np), bd(np);
  std::vector<int32_t> loc(n);
  for (int32_t v = 0; v < n; ++v) {
    loc[v] = (int32_t)mem[part[v]].size();
    mem[part[v]].push_back(v);
  }
  for (int64_t e = 0; e < m; ++e) {
    const int32_t p = part[dst[e]];
    bs[p].push_back(loc[src[e]]);
    bd[p].push_back(loc[dst[e]]);
  }
  ctx->bs_n.assign(np, 0);
  std::vector<int64_t> off(np + 1, 0);
  std::vector<int32_t> flat;
  flat.reserve(n);
  for (int32_t p = 0; p < np; ++p) {
    ctx->bs_n[p] = (int32_t)mem[p].size();
    off[p] = (int64_t)flat.size();
    flat.insert(flat.end(), mem[p].begin(), mem[p].end());
  }
  off[np] = (int64_t)flat.size();
  if (dalloc(&ctx->d_bs_part, n) != hipSuccess || dalloc(&ctx->d_bs_loc, n) != hipSuccess ||
      dalloc(&ctx->d_bs_mem, n) != hipSuccess || dalloc(&ctx->d_bs_n, np) != hipSuccess ||
      dalloc(&ctx->d_bs_off, np + 1) != hipSuccess ||
      dalloc(&ctx->d_bs_pairs, (int64_t)np * np) != hipSuccess)
    return SR_ENOMEM;
  HC(hipMemcpy(ctx->d_bs_part, part, (size_t)n * 4, hipMemcpyHostToDevice));
  HC(hipMemcpy(ctx->d_bs_loc, loc.data(), (size_t)n * 4, hipMemcpyHostToDevice));
  HC(hipMemcpy(ctx->d_bs_mem, flat.data(), (size_t)n * 4, hipMemcpyHostToDevice));
  HC(hipMemcpy(ctx->d_bs_n, ctx->bs_n.data(), (size_t)np * 4, hipMemcpyHostToDevice));
  HC(hipMemcpy(ctx->d_bs_off, off.data(), (size_t)(np + 1) * 8, hipMemcpyHostToDevice));
  ctx->bs_pairs.assign((size_t)np * np, SView{});
  sr_config bc = ctx->cfg;
  bc.mode = SR_DENSE;
  bc.s_prec = SR_S_FP64;
  bc.node_cap = 0;
  bc.edge_cap = 0;
  bc.profile = 0;
  bc.block_store = 0;
  for (int32_t p = 0; p < np; ++p) {
    const int64_t nb = (int64_t)mem[p].size();
    if (nb == 0) continue;
    sr_ctx* b = nullptr;
    sr_status st = init_impl(&b, nb, (int64_t)bs[p].size(), bs[p].data(), bd[p].data(),
                             nullptr, &bc, nullptr, hip_stream, nullptr, nullptr, nullptr);
    if (st != SR_OK) return st;
    st = bs_alloc_pair(ctx, p, p);
    hipError_t e = hipSuccess;
    if (st == SR_OK)
      e = launch_bs_place(ctx->bs_pairs[(int64_t)p * np + p], b->S.d, b->S.ld, nb, ctx->stream);
    if (st == SR_OK && e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    sr_destroy(b);
    if (st != SR_OK) return st;
    HC(e);
  }
  return bs_upload_pairs(ctx);
}

// The fused pass of q deferred blocks (panel ctx->Pb) into the block store: the pairs of
// partition blocks that the blocks' xi and eta supports reach (a pair (p, p') is reached when
// one deferred block has, for one k, a nonzero xi_k entry in p and a nonzero eta_k entry in
// p', or the other way round: its Delta S is sum_k xi_k eta_k^T + eta_k xi_k^T) are
// allocated when new, and the pass adds the chunk's product to every tile of the reached
// pairs; the other deferred blocks' terms are exact zeros there.
sr_status bs_flush(sr_ctx* ctx, int q, int64_t n, int64_t* covered) {
  hipStream_t s = ctx->stream;
  const int32_t np = ctx->bs_np;
  const int nk = ctx->cfg.K + 1;
  const int64_t nf = (int64_t)q * np * nk * 2;
  if (ctx->bs_flags_cap < nf) {
    HC(hipStreamSynchronize(s));
    (void)dfree(ctx->d_bs_flags);
    ctx->d_bs_flags = nullptr;
    ctx->bs_flags_cap = 0;
    if (dalloc(&ctx->d_bs_flags, nf) != hipSuccess) return SR_ENOMEM;
    ctx->bs_flags_cap = nf;
  }
  HC(hipMemsetAsync(ctx->d_bs_flags, 0, (size_t)nf * 4, s));
  HC(launch_bs_touch(ctx->Pb, ctx->pld, ctx->p_rows * ctx->pld, q, nk, n, ctx->d_bs_part, np,
                     ctx->d_bs_flags, s));
  std::vector<uint32_t> f((size_t)nf);
  HC(hipMemcpyAsync(f.data(), ctx->d_bs_flags, (size_t)nf * 4, hipMemcpyDeviceToHost, s));
  HC(hipStreamSynchronize(s));
  std::vector<char> hit((size_t)np * np, 0);
  std::vector<int32_t> xs, es;
  for (int d = 0; d < q; ++d)
    for (int k = 0; k < nk; ++k) {
      xs.clear();
      es.clear();
      for (int32_t p = 0; p < np; ++p) {
        const size_t at = (((size_t)d * np + p) * nk + k) * 2;
        if (f[at]) xs.push_back(p);
        if (f[at + 1]) es.push_back(p);
      }
      for (int32_t a : xs)
        for (int32_t b : es) hit[(size_t)std::min(a, b) * np + std::max(a, b)] = 1;
    }
  bool grew = false;
  std::vector<BsItem> items;
  *covered = 0;
  for (int32_t p = 0; p < np; ++p)
    for (int32_t p2 = p; p2 < np; ++p2) {
      if (!hit[(size_t)p * np + p2] || ctx->bs_n[p] == 0 || ctx->bs_n[p2] == 0) continue;
      // entries of S the pair stands for (both triangles)
      *covered += (int64_t)ctx->bs_n[p] * ctx->bs_n[p2] * (p == p2 ? 1 : 2);
      if (!ctx->bs_pairs[(size_t)p * np + p2].d) {
        const sr_status r = bs_alloc_pair(ctx, p, p2);
        if (r != SR_OK) return r;
        grew = true;
      }
      const int32_t T1 = (ctx->bs_n[p] + 127) / 128, T2 = (ctx->bs_n[p2] + 127) / 128;
      for (int32_t ti = 0; ti < T1; ++ti)
        for (int32_t tj = p == p2 ? ti : 0; tj < T2; ++tj) items.push_back({p, p2, ti, tj});
    }
  if (grew) {
    const sr_status r = bs_upload_pairs(ctx);
    if (r != SR_OK) return r;
  }
  if (items.empty()) return SR_OK;
  const int64_t ni = (int64_t)items.size();
  HC(hipStreamSynchronize(s));  // the previous pass has read the old item list
  if (ctx->bs_items_cap < ni) {
    (void)dfree(ctx->d_bs_items);
    ctx->d_bs_items = nullptr;
    ctx->bs_items_cap = 0;
    const int64_t c = std::max<int64_t>(1024, 2 * ni);
    if (dmalloc((void**)&ctx->d_bs_items, (size_t)c * sizeof(BsItem)) != hipSuccess)
      return SR_ENOMEM;
    ctx->bs_items_cap = c;
  }
  HC(hipMemcpy(ctx->d_bs_items, items.data(), (size_t)ni * sizeof(BsItem),
               hipMemcpyHostToDevice));
  LowRankArgs la{};
  la.S.prec = ctx->cfg.s_prec;
  la.P = ctx->Pb;
  la.pld = ctx->pld;
  la.gstride = ctx->p_rows * ctx->pld;
  la.p_rows = ctx->p_rows;
  la.r = q * ctx->pld;
  const BlockStore bv = bs_view(ctx);
  HC(profiled(ctx, [&]() { return launch_bs_gemm(la, bv, ctx->d_bs_items, ni, s); }));
  return SR_OK;
}

}  // namespace

// Context set-up shared by init_simrank, init_simrank_tree and init_simrank_partitioned. With
// tree_parent, the graph is a spanning forest (tree_parent / tree_depth per node) and S is its
// closed form; with block_part, every edge lies inside a block (block_part per node) and S is
// computed block by block.
static sr_status init_impl(sr_ctx** out, int64_t n, int64_t m, const int32_t* src,
                           const int32_t* dst, const double* weight, const sr_config* cfg_in,
                           const void* S0, void* hip_stream, const int32_t* tree_parent,
                           const int32_t* tree_depth, const int32_t* block_part) {
  if (!out || n <= 0 || m < 0 || (m > 0 && (!src || !dst))) return SR_EINVAL;
  *out = nullptr;
  sr_config cfg;
  if (cfg_in) {
    cfg = *cfg_in;
  } else {
    sr_default_config(&cfg);
  }
  if (!(cfg.C > 0.0 && cfg.C < 1.0) || cfg.K < 0 || cfg.K > 200 || cfg.K_ps < 0 ||
      cfg.s_prec < 0 || cfg.s_prec > 2 || (cfg.mode != SR_DENSE && cfg.mode != SR_COLUMN) ||
      cfg.gamma_form < 0 || cfg.gamma_form > 1 || cfg.batch_chunk < 0 ||
      cfg.batch_chunk > kMaxChunk ||
      cfg.update_prec < 0 || cfg.update_prec > 1 || cfg.block_store < 0 ||
      cfg.block_store > 1 || (cfg.split_rows != 0 && cfg.split_rows < kMedium) ||
      cfg.tile_skip < 0 || cfg.tile_skip > 1)
    return SR_EINVAL;
  if (cfg.block_store && (!block_part || cfg.mode != SR_DENSE)) return SR_EMODE;
  if (cfg.split_rows == 0) cfg.split_rows = kSplitRows;
  // Column mode's default chunk keeps the accumulate passes bounded by matrix-core
  // arithmetic rather than by their read-modify-write of the output: a pass of chunk blocks
  // does chunk 2 (K + 1) / 8 flop per output byte moved, against the ~15 flop per byte where
  // FP64 matrix cores and HBM balance. Measured at n = 1M, K = 10, 8,192 columns, relative
  // to chunk 64 (11.3 GB panel): chunk 24 from 512 columns 0.96 (4.2 GB), chunk 12 0.91
  // (2.2 GB), chunk 1 0.41 (0.26 GB). The panel holds at most 512 + 2 (K + 1) columns of n
  // doubles, a constant multiple of the O(K n) series storage whatever n.
  if (cfg.batch_chunk == 0)
    cfg.batch_chunk = cfg.mode == SR_COLUMN ? std::max(1, (kColumnPanelCols + 2 * cfg.K + 1) /
                                                              (2 * (cfg.K + 1)))
                                            : 64;
  if (cfg.init_max_iter <= 0) cfg.init_max_iter = 400;
  if (cfg.mode == SR_COLUMN && S0) return SR_EINVAL;
  const int64_t node_cap = cfg.node_cap > 0 ? cfg.node_cap : n;
  const int64_t edge_cap = cfg.edge_cap > 0 ? cfg.edge_cap : 2 * m + 1024;
  if (node_cap < n || edge_cap < m || node_cap > ((int64_t)1 << 31) - 64) return SR_ECAPACITY;
  // slot offsets are int32 (see the slot array sizing below)
  if (edge_cap + edge_cap / 4 + 8 * node_cap + edge_cap / 2 + 4096 > ((int64_t)1 << 31) - 1)
    return SR_ECAPACITY;
  // a dense S of more than 2^52 entries (32 PiB) cannot be allocated; refusing here also
  // keeps the byte count below from overflowing
  if (cfg.mode == SR_DENSE && node_cap > ((int64_t)1 << 26)) return SR_ENOMEM;
  for (int64_t e = 0; e < m; ++e) {
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return SR_ERANGE;
    if (src[e] == dst[e]) return SR_ESELF;
  }

  sr_ctx* ctx = new (std::nothrow) sr_ctx();
  if (!ctx) return SR_ENOMEM;
  ctx->cfg = cfg;
  ctx->cfg.node_cap = node_cap;
  ctx->cfg.edge_cap = edge_cap;
  ctx->gemm_variant = cfg.update_prec == SR_UPDATE_FP32 ? kGemmF32 : 0;
  ctx->hin.split = ctx->hout.split = cfg.split_rows;
  ctx->profiling = cfg.profile != 0;
  ctx->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    (void)hipGetLastError();
    delete ctx;
    return SR_EHIP;
  }
  {
    const sr_status rs = resolve_scratch(ctx->device);
    if (rs != SR_OK) {
      delete ctx;
      return rs;
    }
  }
  ctx->node_cap = node_cap;
  ctx->edge_cap = edge_cap;
  ctx->weighted = weight != nullptr;
  ctx->g.n = n;
  ctx->g.m = m;
  ctx->src0.assign(src, src + m);
  ctx->dst0.assign(dst, dst + m);
  if (weight) ctx->w0.assign(weight, weight + m);
  for (int64_t e = 0; e < m; ++e) {
    auto ins = ctx->g.edges.insert(HostGraph::key(src[e], dst[e]));
    if (!ins.second) {
      delete ctx;
      return SR_EEXIST;
    }
  }
  // Slot arrays: a repack of any graph within the capacities fits with room to spare.
  ctx->slot_cap = edge_cap + edge_cap / 4 + 8 * node_cap + edge_cap / 2 + 4096;
  ctx->g.in.build(node_cap, ctx->slot_cap, ctx->dst0, ctx->src0, weight);
  ctx->g.out.build(node_cap, ctx->slot_cap, ctx->src0, ctx->dst0, weight);
  {
    // in-list slot -> initial edge index (build() placed each row's edges in input order)
    ctx->slot_edge0.assign(ctx->g.in.idx.size(), -1);
    std::vector<int32_t> fill(node_cap, 0);
    for (int64_t e = 0; e < m; ++e) {
      const int32_t r = dst[e];
      ctx->slot_edge0[ctx->g.in.start[r] + fill[r]++] = (int32_t)e;
    }
  }

  sr_status st = SR_OK;
#define IC(expr)                      \
  do {                                \
    if ((expr) != hipSuccess) {       \
      sr_destroy(ctx);                \
      return SR_ENOMEM;               \
    }                                 \
  } while (0)
  const int64_t slots = (int64_t)ctx->g.in.idx.size();
  IC(dalloc(&ctx->d_adj[0], node_cap));
  IC(dalloc(&ctx->d_adj[1], node_cap));
  IC(dalloc(&ctx->d_adj[2], slots));
  IC(dalloc(&ctx->d_adj[3], node_cap));
  IC(dalloc(&ctx->d_adj[4], node_cap));
  IC(dalloc(&ctx->d_adj[5], (int64_t)ctx->g.out.idx.size()));
  if (weight) {
    IC(dalloc(&ctx->d_in_w, slots));
    IC(dalloc(&ctx->d_out_w, (int64_t)ctx->g.out.idx.size()));
    IC(dalloc(&ctx->d_W, node_cap));
    std::vector<double>& Wsum = ctx->Wsum;
    Wsum.assign(node_cap, 0.0);
    for (int64_t e = 0; e < m; ++e) Wsum[dst[e]] += weight[e];
    if (hipMemcpy(ctx->d_W, Wsum.data(), node_cap * 8, hipMemcpyHostToDevice) != hipSuccess) {
      sr_destroy(ctx);
      return SR_EHIP;
    }
  }
  // one block's panel width, a multiple of 32: the streaming kernel reads 32 columns per pass
  // (8 per lane group), and passes start at multiples of 32
  ctx->pld = (2 * (cfg.K + 1) + 31) / 32 * 32;
  ctx->W = (int)((node_cap + 31) / 32 + 64);
  IC(dalloc(&ctx->SI, node_cap));
  IC(dalloc(&ctx->Sj, node_cap));
  IC(dalloc(&ctx->QSI, node_cap));
  IC(dalloc(&ctx->zbuf, node_cap));
  IC(dalloc(&ctx->Qz, node_cap));
  IC(dalloc(&ctx->zsum, node_cap));
  IC(dalloc(&ctx->ytmp, node_cap));
  IC(dalloc(&ctx->ylast, node_cap));
  ctx->p_rows = (node_cap + 127) / 128 * 128;
  IC(dalloc(&ctx->P, ctx->p_rows * ctx->pld));
  IC(dalloc(&ctx->pairs, 4 * node_cap));
  IC(dalloc(&ctx->suppI, ctx->W));
  IC(dalloc(&ctx->suppJ, ctx->W));
  IC(dalloc(&ctx->Abits, (int64_t)(cfg.K + 1) * ctx->W));
  IC(dalloc(&ctx->Bbits, (int64_t)(cfg.K + 1) * ctx->W));
  IC(dalloc(&ctx->Ahat, ctx->W));
  IC(dalloc(&ctx->Bhat, ctx->W));
  IC(dalloc(&ctx->rowlist, node_cap));
  IC(dalloc(&ctx->rowlist2, node_cap));
  IC(dalloc(&ctx->d_cnt, 8));
  IC(dalloc(&ctx->d_max, 1));
  IC(dalloc(&ctx->d_sum, 4));
  IC(dalloc(&ctx->d_mm, 4));
  IC(hipHostMalloc((void**)&ctx->h_cnt, 8 * sizeof(int64_t), hipHostMallocDefault));
  IC(hipHostMalloc((void**)&ctx->h_max, sizeof(unsigned long long), hipHostMallocDefault));
  if (hipMemset(ctx->P, 0, (size_t)ctx->p_rows * ctx->pld * 8) != hipSuccess ||
      hipMemset(ctx->Ahat, 0, (size_t)ctx->W * 4) != hipSuccess ||
      hipMemset(ctx->Bhat, 0, (size_t)ctx->W * 4) != hipSuccess ||
      hipMemset(ctx->Abits, 0, (size_t)(cfg.K + 1) * ctx->W * 4) != hipSuccess ||
      hipMemset(ctx->Bbits, 0, (size_t)(cfg.K + 1) * ctx->W * 4) != hipSuccess ||
      hipMemset(ctx->suppI, 0, (size_t)ctx->W * 4) != hipSuccess ||
      hipMemset(ctx->suppJ, 0, (size_t)ctx->W * 4) != hipSuccess) {
    sr_destroy(ctx);
    return SR_EHIP;
  }
  st = upload_graph(ctx);
  for (int64_t r = 0; r < node_cap && st == SR_OK; ++r) {
    heavy_touch(ctx->hin, ctx->g.in, (int32_t)r);
    heavy_touch(ctx->hout, ctx->g.out, (int32_t)r);
  }
  if (st == SR_OK) st = heavy_refresh(ctx);
  if (st != SR_OK) {
    sr_destroy(ctx);
    return st;
  }

  if (cfg.mode == SR_COLUMN) {
    const int Kp = cfg.K_ps > 0 ? cfg.K_ps : cfg.K;
    IC(dalloc(&ctx->xs, (int64_t)(Kp + 1) * 2 * node_cap));
    IC(dalloc(&ctx->xd, 4 * node_cap));
    *out = ctx;
    return SR_OK;
  }

  // Dense S with leading dimension node_cap rounded to 64; rows/cols past n stay zero.
  const int64_t ld = (node_cap + 63) / 64 * 64;
  ctx->S.prec = cfg.s_prec;
  ctx->S.ld = ld;
  const size_t cells = (size_t)node_cap * (size_t)ld;
  if (cfg.block_store) {
    // no dense store: S lives in the block pairs (block_store_init below)
  } else if (cfg.s_prec == SR_S_FP64) {
    IC(dmalloc((void**)&ctx->S_mem[0], cells * 8));
    ctx->S.d = (double*)ctx->S_mem[0];
    IC(hipMemset(ctx->S_mem[0], 0, cells * 8));
  } else if (cfg.s_prec == SR_S_FP32_HILO) {
    IC(dmalloc((void**)&ctx->S_mem[0], cells * 8));
    ctx->S.hl = (float2*)ctx->S_mem[0];
    IC(hipMemset(ctx->S_mem[0], 0, cells * 8));
  } else {
    IC(dmalloc((void**)&ctx->S_mem[0], cells * 4));
    ctx->S.hi = (float*)ctx->S_mem[0];
    IC(hipMemset(ctx->S_mem[0], 0, cells * 4));
  }

  if (block_part && cfg.block_store) {
    const sr_status bst = block_store_init(ctx, n, m, src, dst, block_part, hip_stream);
    if (bst != SR_OK) {
      sr_destroy(ctx);
      return bst;
    }
    ctx->updated = false;
    *out = ctx;
    return SR_OK;
  }

  if (block_part) {
    // S of the blocks' own edges, block by block (Example 1.1): each block's fixed point on a
    // context of its own nodes (float64), placed on the diagonal of the store
    int32_t np = 0;
    for (int64_t v = 0; v < n; ++v) np = std::max(np, block_part[v] + 1);
    std::vector<std::vector<int32_t>> mem(np), bs(np), bd(np);
    std::vector<int32_t> loc(n);
    for (int32_t v = 0; v < n; ++v) {
      loc[v] = (int32_t)mem[block_part[v]].size();
      mem[block_part[v]].push_back(v);
    }
    for (int64_t e = 0; e < m; ++e) {
      const int32_t p = block_part[dst[e]];
      bs[p].push_back(loc[src[e]]);
      bd[p].push_back(loc[dst[e]]);
    }
    sr_config bc = cfg;
    bc.mode = SR_DENSE;
    bc.s_prec = SR_S_FP64;
    bc.node_cap = 0;
    bc.edge_cap = 0;
    bc.profile = 0;
    int32_t* dg = nullptr;
    hipError_t e = dmalloc((void**)&dg, (size_t)n * 4);
    sr_status bst = SR_OK;
    for (int32_t p = 0; p < np && e == hipSuccess && bst == SR_OK; ++p) {
      const int64_t nb = (int64_t)mem[p].size();
      if (nb == 0) continue;
      sr_ctx* b = nullptr;
      bst = init_impl(&b, nb, (int64_t)bs[p].size(), bs[p].data(), bd[p].data(), nullptr, &bc,
                      nullptr, hip_stream, nullptr, nullptr, nullptr);
      if (bst != SR_OK) break;
      e = hipMemcpy(dg, mem[p].data(), (size_t)nb * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = launch_place_block(ctx->S, dg, nb, b->S.d, b->S.ld, ctx->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      sr_destroy(b);
    }
    (void)dfree(dg);
    if (bst != SR_OK || e != hipSuccess) {
      sr_destroy(ctx);
      return bst != SR_OK ? bst : SR_EHIP;
    }
    ctx->updated = false;
    *out = ctx;
    return SR_OK;
  }

  if (tree_parent) {
    // S of the forest by Example 1.2's closed form, written straight into the store
    int32_t *dp = nullptr, *dd = nullptr;
    hipError_t e = dmalloc((void**)&dp, (size_t)n * 4);
    if (e == hipSuccess) e = dmalloc((void**)&dd, (size_t)n * 4);
    if (e == hipSuccess) e = hipMemcpy(dp, tree_parent, (size_t)n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dd, tree_depth, (size_t)n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_tree_init(ctx->S, n, dp, dd, cfg.C, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)dfree(dp);
    (void)dfree(dd);
    if (e != hipSuccess) {
      sr_destroy(ctx);
      return SR_EHIP;
    }
    ctx->updated = false;
    *out = ctx;
    return SR_OK;
  }

  // Initial S: copy S0, or iterate S <- C Q S Q^T + (1 - C) I in float64 (eq (03a)):
  //   T = Q S (row gather), U = T^T, S' = C Q U + (1 - C) I; S symmetric so U = S Q^T.
  const int64_t ldi = (n + 63) / 64 * 64;
  double *A = nullptr, *B = nullptr, *T = nullptr;
  IC(dalloc(&A, n * ldi));
  if (S0) {
    // S0 has leading dimension n; re-pitch into ldi
    if (hipMemcpy2D(A, ldi * 8, S0, n * 8, n * 8, n, hipMemcpyDeviceToDevice) != hipSuccess) {
      (void)dfree(A);
      sr_destroy(ctx);
      return SR_EHIP;
    }
  } else {
    IC(dalloc(&B, n * ldi));
    IC(dalloc(&T, n * ldi));
    hipError_t e = hipMemsetAsync(A, 0, (size_t)n * ldi * 8, ctx->stream);
    if (e == hipSuccess) e = launch_fill_diag(A, n, ldi, 1.0 - cfg.C, ctx->stream);
    for (int it = 0; it < cfg.init_max_iter && e == hipSuccess; ++it) {
      e = hipMemsetAsync(ctx->d_max, 0, 8, ctx->stream);
      if (e == hipSuccess) e = launch_spmm_rows(devq(ctx), n, A, T, 1.0, 0.0, nullptr, nullptr,
                                                ctx->stream);
      if (e == hipSuccess) e = launch_transpose(n, T, B, ctx->stream);
      if (e == hipSuccess) e = launch_spmm_rows(devq(ctx), n, B, T, cfg.C, 1.0 - cfg.C, A,
                                                ctx->d_max, ctx->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(ctx->h_max, ctx->d_max, 8, hipMemcpyDeviceToHost,
                                              ctx->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      std::swap(A, T);
      double step;
      memcpy(&step, ctx->h_max, 8);
      if (step <= cfg.init_tol) break;
    }
    if (e != hipSuccess) {
      (void)dfree(A);
      (void)dfree(B);
      (void)dfree(T);
      sr_destroy(ctx);
      return SR_EHIP;
    }
  }
  // The two gathers of an iteration sum in different orders for (a, b) and (b, a); the
  // stored S is made exactly symmetric, (A + A^T) / 2, which the mirrored updates keep.
  hipError_t e = hipSuccess;
  if (B) e = launch_transpose(n, A, B, ctx->stream);
  if (e == hipSuccess) e = launch_to_store(ctx->S, n, A, ctx->stream, B);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)dfree(A);
  (void)dfree(B);
  (void)dfree(T);
  if (e != hipSuccess) {
    sr_destroy(ctx);
    return SR_EHIP;
  }
  ctx->updated = false;
  *out = ctx;
  return SR_OK;
#undef IC
}

sr_status init_simrank(sr_ctx** out, int64_t n, int64_t m, const int32_t* src,
                       const int32_t* dst, const double* weight, const sr_config* cfg_in,
                       const void* S0, void* hip_stream) {
  return init_impl(out, n, m, src, dst, weight, cfg_in, S0, hip_stream, nullptr, nullptr,
                   nullptr);
}

sr_status init_simrank_tree(sr_ctx** out, int64_t n, int64_t m, const int32_t* src,
                            const int32_t* dst, const sr_config* cfg_in, void* hip_stream,
                            sr_batch_stats* stats) {
  if (!out || n <= 0 || m < 0 || (m > 0 && (!src || !dst))) return SR_EINVAL;
  *out = nullptr;
  sr_config cfg;
  if (cfg_in) {
    cfg = *cfg_in;
  } else {
    sr_default_config(&cfg);
  }
  if (cfg.mode != SR_DENSE) return SR_EMODE;
  for (int64_t e = 0; e < m; ++e) {
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return SR_ERANGE;
    if (src[e] == dst[e]) return SR_ESELF;
  }
  if (cfg.edge_cap <= 0) cfg.edge_cap = 2 * m + 1024;
  // Breadth-first spanning forest (Example 1.2): nodes without in-edges are roots first, then
  // any node not reached yet, both in ascending id; out-neighbours scanned in ascending id.
  std::vector<int64_t> ostart(n + 1, 0);
  std::vector<int32_t> indeg(n, 0);
  for (int64_t e = 0; e < m; ++e) {
    ++ostart[src[e] + 1];
    ++indeg[dst[e]];
  }
  for (int64_t v = 0; v < n; ++v) ostart[v + 1] += ostart[v];
  std::vector<int32_t> onb(m);
  {
    std::vector<int64_t> fill(ostart.begin(), ostart.end() - 1);
    for (int64_t e = 0; e < m; ++e) onb[fill[src[e]]++] = dst[e];
    for (int64_t v = 0; v < n; ++v) std::sort(onb.begin() + ostart[v], onb.begin() + ostart[v + 1]);
  }
  std::vector<int32_t> parent(n, -1), depth(n, 0), queue;
  std::vector<char> seen(n, 0);
  queue.reserve(n);
  auto grow = [&](int32_t r) {
    if (seen[r]) return;
    seen[r] = 1;
    size_t head = queue.size();
    queue.push_back(r);
    while (head < queue.size()) {
      const int32_t u = queue[head++];
      for (int64_t p = ostart[u]; p < ostart[u + 1]; ++p) {
        const int32_t v = onb[p];
        if (!seen[v]) {
          seen[v] = 1;
          parent[v] = u;
          depth[v] = depth[u] + 1;
          queue.push_back(v);
        }
      }
    }
  };
  for (int32_t v = 0; v < n; ++v)
    if (indeg[v] == 0) grow(v);
  for (int32_t v = 0; v < n; ++v) grow(v);
  // forest edges parent[v] -> v (by v); the other edges keep the caller's order
  std::vector<int32_t> ts, td, rs, rd;
  for (int32_t v = 0; v < n; ++v)
    if (parent[v] >= 0) {
      ts.push_back(parent[v]);
      td.push_back(v);
    }
  for (int64_t e = 0; e < m; ++e)
    if (parent[dst[e]] != src[e]) {
      rs.push_back(src[e]);
      rd.push_back(dst[e]);
    }
  if ((int64_t)(ts.size() + rs.size()) != m) return SR_EEXIST;  // a forest edge given twice
  sr_ctx* ctx = nullptr;
  sr_status st = init_impl(&ctx, n, (int64_t)ts.size(), ts.data(), td.data(), nullptr, &cfg,
                           nullptr, hip_stream, parent.data(), depth.data(), nullptr);
  if (st != SR_OK) return st;
  std::vector<int8_t> ops(rs.size(), 1);
  st = apply_batch(ctx, (int64_t)rs.size(), rs.data(), rd.data(), ops.data(), stats);
  if (st != SR_OK) {
    sr_destroy(ctx);
    return st;
  }
  *out = ctx;
  return SR_OK;
}

sr_status sr_partition(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                       int32_t parts, int32_t* part_out) {
  if (n <= 0 || m < 0 || parts < 1 || !part_out || (m > 0 && (!src || !dst))) return SR_EINVAL;
  for (int64_t e = 0; e < m; ++e)
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return SR_ERANGE;
  // undirected neighbour lists, ascending and without repeats
  std::vector<int64_t> start(n + 1, 0);
  for (int64_t e = 0; e < m; ++e) {
    ++start[src[e] + 1];
    ++start[dst[e] + 1];
  }
  for (int64_t v = 0; v < n; ++v) start[v + 1] += start[v];
  std::vector<int32_t> nb(2 * m);
  {
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t e = 0; e < m; ++e) {
      nb[fill[src[e]]++] = dst[e];
      nb[fill[dst[e]]++] = src[e];
    }
  }
  std::vector<int64_t> len(n);
  for (int64_t v = 0; v < n; ++v) {
    auto b = nb.begin() + start[v], e = nb.begin() + start[v + 1];
    std::sort(b, e);
    len[v] = std::unique(b, e) - b;
  }
  // blocks of at most ceil(n / parts) nodes, grown breadth first from the smallest
  // unassigned id; a full block stops at once, a dry search continues from the next seed
  const int64_t cap = (n + parts - 1) / parts;
  for (int64_t v = 0; v < n; ++v) part_out[v] = -1;
  std::vector<int32_t> queue;
  queue.reserve(n);
  int32_t p = 0;
  int64_t size = 0, next = 0;
  while (true) {
    while (next < n && part_out[next] >= 0) ++next;
    if (next == n) break;
    part_out[next] = p;
    ++size;
    queue.clear();
    queue.push_back((int32_t)next);
    bool full = size == cap;
    for (size_t h = 0; h < queue.size() && !full; ++h) {
      const int32_t u = queue[h];
      for (int64_t q = start[u]; q < start[u] + len[u]; ++q) {
        const int32_t v = nb[q];
        if (part_out[v] < 0) {
          part_out[v] = p;
          ++size;
          queue.push_back(v);
          if (size == cap) {
            full = true;
            break;
          }
        }
      }
    }
    if (full) {
      ++p;
      size = 0;
    }
  }
  return SR_OK;
}

sr_status init_simrank_partitioned(sr_ctx** out, int64_t n, int64_t m, const int32_t* src,
                                   const int32_t* dst, const int32_t* part,
                                   const sr_config* cfg_in, void* hip_stream,
                                   sr_batch_stats* stats) {
  if (!out || n <= 0 || m < 0 || !part || (m > 0 && (!src || !dst))) return SR_EINVAL;
  *out = nullptr;
  sr_config cfg;
  if (cfg_in) {
    cfg = *cfg_in;
  } else {
    sr_default_config(&cfg);
  }
  if (cfg.mode != SR_DENSE) return SR_EMODE;
  for (int64_t v = 0; v < n; ++v)
    if (part[v] < 0 || part[v] >= n) return SR_ERANGE;
  for (int64_t e = 0; e < m; ++e) {
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return SR_ERANGE;
    if (src[e] == dst[e]) return SR_ESELF;
  }
  if (cfg.edge_cap <= 0) cfg.edge_cap = 2 * m + 1024;
  std::vector<int32_t> is, id, cs, cd;
  for (int64_t e = 0; e < m; ++e) {
    if (part[src[e]] == part[dst[e]]) {
      is.push_back(src[e]);
      id.push_back(dst[e]);
    } else {
      cs.push_back(src[e]);
      cd.push_back(dst[e]);
    }
  }
  sr_ctx* ctx = nullptr;
  sr_status st = init_impl(&ctx, n, (int64_t)is.size(), is.data(), id.data(), nullptr, &cfg,
                           nullptr, hip_stream, nullptr, nullptr, part);
  if (st != SR_OK) return st;
  std::vector<int8_t> ops(cs.size(), 1);
  st = apply_batch(ctx, (int64_t)cs.size(), cs.data(), cd.data(), ops.data(), stats);
  if (st != SR_OK) {
    sr_destroy(ctx);
    return st;
  }
  *out = ctx;
  return SR_OK;
}

}  // extern "C"

// One unit update: op = +1 inserts i -> j (weight w_new on a weighted graph), -1 deletes it;
// reweight (weighted graphs) changes the weight of the existing edge from w_old to w_new.
static sr_status unit_update(sr_ctx* ctx, int32_t i, int32_t j, int32_t op, double w_old,
                             double w_new, bool reweight, sr_update_stats* stats) {
  const int64_t n = ctx->g.n;
  if (i < 0 || j < 0) return SR_ERANGE;
  if (i == j) return SR_ESELF;
  int case_id;
  if (i < n && j < n) {
    case_id = 0;
  } else if (i < n && j == n) {
    case_id = 1;
  } else if (i == n && j < n) {
    case_id = 2;
  } else if (i == n && j == n + 1) {
    case_id = 3;
  } else {
    return SR_ERANGE;
  }
  if (op < 0 && case_id != 0) return SR_ENOENT;
  if (ctx->bstore) return SR_EMODE;  // the block store takes batches (apply_batch) only
  if (case_id == 0) {
    const bool has = ctx->g.has(i, j);
    if (op > 0 && has && !reweight) return SR_EEXIST;
    if ((op < 0 || reweight) && !has) return SR_ENOENT;
  }
  if (ctx->weighted && ctx->cfg.mode == SR_COLUMN) return SR_EMODE;
  const int64_t n_new = n + (case_id == 3 ? 2 : (case_id == 0 ? 0 : 1));
  if (n_new > ctx->node_cap) return SR_ECAPACITY;
  if (op > 0 && !reweight && ctx->g.m + 1 > ctx->edge_cap) return SR_ECAPACITY;
  if (op > 0 && !reweight && !graph_fits(ctx, {{i, j}})) return SR_ECAPACITY;

  ctx->last_case = -1;
  ctx->last_r = 0;
  if (ctx->cfg.mode == SR_COLUMN) {
    // Algorithm 7 (column method): S is not stored; the old columns an update needs come
    // from PartialSim on the current graph, and the update's Delta S columns are kept in
    // factored form for query_columns / query_column(SR_COL_DELTA).
    hipStream_t s = ctx->stream;
    const double C = ctx->cfg.C;
    const int K = ctx->cfg.K;
    IdList li, lj;
    li.count = lj.count = 1;
    li.id[0] = i;
    lj.id[0] = j;
    if (stats) {
      memset(stats, 0, sizeof(*stats));
      HC(hipMemsetAsync(ctx->d_max, 0, 8, s));
    }
    const int64_t dj = ctx->g.in.len[j < n ? j : 0] * (j < n ? 1 : 0);
    double xi0 = C;
    sr_status r = SR_OK;
    if (case_id == 0 || case_id == 2) {
      GammaArgs ga{};
      ga.op = op;
      ga.j = j;
      ga.delta = 1;
      ga.dj = dj;
      ga.C = C;
      if (case_id == 0) {
        // Table 2 row C0 (Theorem 3 insertion, Theorem 9 deletion): S[:, i], S[:, j]
        r = partial_sim2(ctx, li, lj, ctx->SI, ctx->Sj);
        if (r != SR_OK) return r;
        HC(launch_spmv_q(devq(ctx), heavy_args(ctx->hin), n, ctx->SI, ctx->QSI, 1.0, s));
        ga.kind = 0;
        ga.I = li;
      } else {
        // C2: the new source joins as an isolated node, then Table 2 row C2 (eq (60)) on
        // the grown graph; S[:, j] on it is zero at the new node
        ctx->g.n = n_new;
        r = partial_sim(ctx, lj, ctx->Sj);
        if (r != SR_OK) return r;
        ga.kind = 2;
        xi0 = C / (double)(dj + 1);
      }
      ga.xi0 = xi0;
      HC(launch_gamma(ga, n_new, ctx->SI, ctx->Sj, ctx->QSI, nullptr, nullptr, ctx->P, ctx->pld,
                      stats ? ctx->d_max : nullptr, s));
      r = edit_graph(ctx, {{i, j}}, op);
      if (r != SR_OK) return r;
      for (int k = 0; k < K; ++k)
        HC(launch_series_step(devq(ctx), heavy_args(ctx->hin), n_new, ctx->P, ctx->pld, k, C,
                              1.0, nullptr, s, ctx->pairs, ctx->node_cap));
      ctx->last_r = 2 * (K + 1);
    } else if (case_id == 1) {
      // Theorem 8 / Table 2 row C1: the new sink's column y = C Q S[:, i] on the old graph,
      // its diagonal C S_ii + 1 - C; every other column only gains its entry y[x] at j
      r = partial_sim(ctx, li, ctx->SI);
      if (r != SR_OK) return r;
      HC(launch_spmv_q(devq(ctx), heavy_args(ctx->hin), n, ctx->SI, ctx->ylast, C, s));
      HC(launch_c1_corner(ctx->ylast, j, ctx->SI, li, C, s));
      ctx->g.n = n_new;
      r = edit_graph(ctx, {{i, j}}, +1);
      if (r != SR_OK) return r;
    } else {
      // Algorithm 5 / Table 2 row C3 with one source: two new nodes, diagonals only
      ctx->g.n = n_new;
      r = edit_graph(ctx, {{i, j}}, +1);
      if (r != SR_OK) return r;
    }
    ctx->last_case = case_id;
    ctx->last_i = i;
    ctx->last_j = j;
    ctx->last_vi = 1.0 - C;
    ctx->last_vj = (1.0 - C) * (1.0 + C);
    if (stats) {
      stats->case_id = case_id;
      stats->op = op;
      stats->d_j = dj;
      stats->n_after = n_new;
      if (case_id == 0 || case_id == 2) {
        HC(hipMemcpyAsync(ctx->h_max, ctx->d_max, 8, hipMemcpyDeviceToHost, s));
        HC(hipStreamSynchronize(s));
        double gmax;
        memcpy(&gmax, ctx->h_max, 8);
        stats->bound = 2.0 * xi0 * pow(C, K + 1) / (1.0 - C) * gmax;
      } else {
        HC(hipStreamSynchronize(s));
      }
    }
    return SR_OK;
  }

  if (stats) memset(stats, 0, sizeof(*stats));
  sr_status r = SR_OK;
  const double C = ctx->cfg.C;
  if (case_id == 0) {
    // weighted graphs: the scale a of Delta Q = e_j a (e_i - Q[j, :])^T; the two cases
    // where row j of Q is empty before or after take the weight-free unweighted forms
    double alpha = 0.0;
    if (ctx->weighted) {
      const double Wj = ctx->Wsum[j];
      const int64_t dj = ctx->g.in.len[j];
      if (reweight)
        alpha = (w_new - w_old) / (Wj + (w_new - w_old));
      else if (op > 0 && dj > 0)
        alpha = w_new / (Wj + w_new);
      else if (op < 0 && dj > 1)
        alpha = -w_old / (Wj - w_old);
    }
    r = lowrank_block(ctx, 0, op, {i}, j, n, stats, nullptr, nullptr, alpha, reweight, w_new);
  } else if (case_id == 1) {
    ctx->g.n = n_new;
    r = c1_block(ctx, {i}, j, n, nullptr, nullptr, w_new);
    ctx->last_r = 0;
  } else if (case_id == 2) {
    ctx->g.n = n_new;
    const double alpha = ctx->weighted ? w_new / (ctx->Wsum[j] + w_new) : 0.0;
    r = set_diags(ctx, {{i, 1.0 - C}});
    if (r == SR_OK)
      r = lowrank_block(ctx, 2, +1, {i}, j, n_new, stats, nullptr, nullptr, alpha, false, w_new);
  } else {
    ctx->g.n = n_new;
    r = c3_block(ctx, {i}, j, w_new);
    ctx->last_r = 0;
  }
  if (r != SR_OK) return r;
  ctx->last_case = case_id;
  ctx->last_i = i;
  ctx->last_j = j;
  ctx->last_vi = 1.0 - C;
  ctx->last_vj = (1.0 - C) * (1.0 + C);
  if (stats) {
    stats->case_id = case_id;
    stats->op = op;
    stats->n_after = n_new;
    if (case_id == 1 || case_id == 3) {
      stats->d_j = 0;
      stats->pairs = case_id == 1 ? 2 * n + 1 : 2;
      HC(hipStreamSynchronize(ctx->stream));
    }
  }
  return SR_OK;
}

extern "C" {

sr_status apply_edge_update(sr_ctx* ctx, int32_t i, int32_t j, int32_t op,
                            sr_update_stats* stats) {
  if (!valid_ctx(ctx)) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  if (op != 1 && op != -1) return SR_EINVAL;
  double w_old = 0.0;
  if (op < 0 && ctx->weighted && i >= 0 && j >= 0 && i < ctx->g.n && j < ctx->g.n) {
    const int32_t p = ctx->g.in.find(j, i);
    if (p >= 0) w_old = ctx->g.in.w[ctx->g.in.start[j] + p];
  }
  return unit_update(ctx, i, j, op, w_old, op > 0 ? 1.0 : 0.0, false, stats);
}

sr_status apply_weight_update(sr_ctx* ctx, int32_t i, int32_t j, double w,
                              sr_update_stats* stats) {
  if (!valid_ctx(ctx)) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  if (!ctx->weighted) return SR_EMODE;
  if (!(w >= 0.0) || !std::isfinite(w)) return SR_EINVAL;
  const int64_t n = ctx->g.n;
  if (i < 0 || j < 0) return SR_ERANGE;
  if (i == j) return SR_ESELF;
  double w_old = 0.0;
  if (i < n && j < n) {
    const int32_t p = ctx->g.in.find(j, i);
    if (p >= 0) w_old = ctx->g.in.w[ctx->g.in.start[j] + p];
  }
  if (w_old == 0.0 && w == 0.0) return SR_ENOENT;
  if (w == w_old) {
    if (stats) {
      memset(stats, 0, sizeof(*stats));
      stats->n_after = n;
    }
    return SR_OK;
  }
  if (w_old == 0.0) return unit_update(ctx, i, j, +1, 0.0, w, false, stats);
  if (w == 0.0) return unit_update(ctx, i, j, -1, w_old, 0.0, false, stats);
  return unit_update(ctx, i, j, +1, w_old, w, true, stats);
}

// ------------------------------------------------------------------------------ batches

}  // extern "C"

namespace {

struct Block {
  int case_id;
  int op;
  int32_t j;
  int64_t dj;
  std::vector<int32_t> I;
};

// Algorithm 6 planning (section 8). Returns SR_OK and the blocks, or a validation status.
sr_status plan_batch(const sr_ctx* ctx, int64_t cnt, const int32_t* bi, const int32_t* bj,
                     const int8_t* bo, std::vector<Block>& plan, int64_t& n_new,
                     int64_t& net_edges) {
  const int64_t n = ctx->g.n;
  std::map<std::pair<int32_t, int32_t>, int> net;  // (j, i) -> count, ordered by sink
  for (int64_t e = 0; e < cnt; ++e) {
    if (bo[e] != 1 && bo[e] != -1) return SR_EINVAL;
    if (bi[e] < 0 || bj[e] < 0) return SR_ERANGE;
    if (bi[e] == bj[e]) return SR_ESELF;
    net[{bj[e], bi[e]}] += bo[e];
  }
  std::set<int32_t> newids;
  std::vector<std::pair<int32_t, int32_t>> plus, minus;  // (j, i)
  for (auto& kv : net) {
    const int32_t j = kv.first.first, i = kv.first.second;
    if (kv.second > 1) return SR_EEXIST;
    if (kv.second < -1) return SR_ENOENT;
    if (i >= n) newids.insert(i);
    if (j >= n) newids.insert(j);
  }
  for (int64_t e = 0; e < cnt; ++e) {
    if (bi[e] >= n) newids.insert(bi[e]);
    if (bj[e] >= n) newids.insert(bj[e]);
  }
  n_new = n + (int64_t)newids.size();
  if (!newids.empty() && (*newids.begin() != n || *newids.rbegin() != n_new - 1))
    return SR_ERANGE;
  if (n_new > ctx->node_cap) return SR_ECAPACITY;
  int64_t ins = 0;
  for (auto& kv : net) {
    const int32_t j = kv.first.first, i = kv.first.second;
    const bool old_edge = (i < n && j < n) && ctx->g.has(i, j);
    if (kv.second == 1) {
      if (old_edge) return SR_EEXIST;
      plus.push_back({j, i});
      ++ins;
    } else if (kv.second == -1) {
      if (!old_edge) return SR_ENOENT;
      minus.push_back({j, i});
    }
  }
  if (ctx->g.m + ins > ctx->edge_cap) return SR_ECAPACITY;
  {
    std::vector<std::pair<int32_t, int32_t>> ie;
    ie.reserve(plus.size());
    for (const auto& ji : plus) ie.push_back({ji.second, ji.first});
    if (!graph_fits(ctx, ie)) return SR_ECAPACITY;
  }
  net_edges = (int64_t)(plus.size() + minus.size());

  std::vector<int64_t> deg_change;  // tracked lazily through a map
  std::map<int32_t, int64_t> dmod;
  auto degree = [&](int32_t j) -> int64_t {
    int64_t d = j < n ? ctx->g.in.len[j] : 0;
    auto it = dmod.find(j);
    return d + (it == dmod.end() ? 0 : it->second);
  };
  // one block per sink (and per old / new source split of an insertion block): Table 2
  // applies the whole block as one rank-one update, whatever its size
  auto push_block = [&](int case_id, int op, int32_t j, std::vector<int32_t>& I) {
    Block b;
    b.case_id = case_id;
    b.op = op;
    b.j = j;
    b.dj = degree(j);
    b.I = I;
    dmod[j] += op * (int64_t)b.I.size();
    plan.push_back(b);
  };
  // deletion blocks, sinks ascending
  for (size_t a = 0; a < minus.size();) {
    size_t b = a;
    std::vector<int32_t> I;
    while (b < minus.size() && minus[b].first == minus[a].first) I.push_back(minus[b++].second);
    push_block(0, -1, minus[a].first, I);
    a = b;
  }
  // insertion blocks, sinks ascending; split by source existence at processing time
  std::set<int32_t> created;
  auto exists = [&](int32_t v) { return v < n || created.count(v) != 0; };
  for (size_t a = 0; a < plus.size();) {
    size_t b = a;
    const int32_t j = plus[a].first;
    std::vector<int32_t> old_src, new_src;
    while (b < plus.size() && plus[b].first == j) {
      const int32_t i = plus[b++].second;
      (exists(i) ? old_src : new_src).push_back(i);
    }
    if (!old_src.empty()) {
      push_block(exists(j) ? 0 : 1, 1, j, old_src);
      created.insert(j);
    }
    if (!new_src.empty()) {
      push_block(exists(j) ? 2 : 3, 1, j, new_src);
      created.insert(j);
      for (int32_t i : new_src) created.insert(i);
    }
    a = b;
  }
  return SR_OK;
}

}  // namespace

extern "C" {

sr_status apply_batch(sr_ctx* ctx, int64_t cnt, const int32_t* bi, const int32_t* bj,
                      const int8_t* bo, sr_batch_stats* stats) {
  if (!valid_ctx(ctx)) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  if (cnt < 0 || (cnt > 0 && (!bi || !bj || !bo))) return SR_EINVAL;
  if (ctx->cfg.mode != SR_DENSE || ctx->weighted) return SR_EMODE;
  std::vector<Block> plan;
  int64_t n_new = 0, net_edges = 0;
  sr_status r = plan_batch(ctx, cnt, bi, bj, bo, plan, n_new, net_edges);
  if (r != SR_OK) return r;
  const int64_t n_old = ctx->g.n;
  if (ctx->bstore) {
    // the block store takes fused passes of blocks between existing nodes only
    if (n_new != n_old || !ctx->cfg.fused_batch || ctx->cfg.gamma_form != SR_GAMMA_CLOSED)
      return SR_EMODE;
    for (const Block& b : plan)
      if (b.case_id != 0) return SR_EMODE;
  }
  const double C = ctx->cfg.C;
  // New nodes start as isolated nodes (SimRank 1 - C on the diagonal, 0 elsewhere); a block
  // that creates one then writes its case's values.
  HC(launch_diag_range(ctx->S, n_old, n_new, 1.0 - C, ctx->stream));
  ctx->g.n = n_new;
  int64_t pairs = 0, lowrank = 0, bc[4] = {0, 0, 0, 0};
  // Fused form: low-rank blocks write their pairs side by side into Pb; every batch_chunk
  // blocks (and at the end) one pass adds all of them to S (rank 2 (K+1) x blocks).
  const bool fused = ctx->cfg.fused_batch != 0 && ctx->cfg.gamma_form == SR_GAMMA_CLOSED;
  const int chunk = ctx->cfg.batch_chunk;
  const int pld_all = ctx->pld * chunk;
  if (fused && !ctx->Pb) {
    if (dalloc(&ctx->Pb, ctx->p_rows * (int64_t)pld_all) != hipSuccess ||
        dalloc(&ctx->wts, 2 * (int64_t)pld_all) != hipSuccess)
      return SR_ENOMEM;
    // padding columns of each block's segment are never written and must read as zero
    HC(hipMemsetAsync(ctx->Pb, 0, (size_t)ctx->p_rows * pld_all * 8, ctx->stream));
  }
  int q = 0;  // deferred blocks in the current chunk
  int passes = 0;
  std::vector<int> pass_blocks;  // deferred blocks of each dense fused pass
  if (fused && !ctx->bstore) {
    // per pass: the reached-node list's length (at most one pass per plan block, plus one)
    if (!ctx->d_act) {
      if (dalloc(&ctx->d_act, ctx->node_cap) != hipSuccess ||
          dalloc(&ctx->d_act_bits, (int64_t)ctx->W) != hipSuccess)
        return SR_ENOMEM;
    }
    const int64_t need = (int64_t)plan.size() + 1;
    if (ctx->act_cnt_cap < need) {
      HC(hipStreamSynchronize(ctx->stream));
      (void)dfree(ctx->d_act_cnt);
      ctx->d_act_cnt = nullptr;
      ctx->act_cnt_cap = 0;
      const int64_t c = std::max<int64_t>(256, 2 * need);
      if (dalloc(&ctx->d_act_cnt, c) != hipSuccess) return SR_ENOMEM;
      ctx->act_cnt_cap = c;
    }
  }
  // Tile skipping (float64 matrix cores): flags of one pass (chunk blocks x tiles of the node
  // range) and, per low-rank block of the batch, the skipped positions of its counted k-steps.
  const int steps_all = ctx->pld / 4;
  const int steps_used = (ctx->cfg.K + 2) / 2;  // k-steps holding series columns
  const bool tskip = fused && !ctx->bstore && ctx->cfg.tile_skip != 0 &&
                     ctx->gemm_variant != kGemmF32 && steps_all <= 32;
  int64_t tf_ld = 0;
  int64_t skip_blocks = 0;  // low-rank blocks of the batch's dense passes so far
  if (tskip) {
    tf_ld = (n_new + kTileRows - 1) / kTileRows;
    const int64_t nf = (int64_t)chunk * tf_ld;
    int64_t nlow = 0;
    for (const Block& b : plan) nlow += (b.case_id == 0 || b.case_id == 2);
    const int64_t ns = std::max<int64_t>(1, nlow * steps_used);
    if (ctx->tflags_cap < nf || ctx->skip_cap < ns) {
      HC(hipStreamSynchronize(ctx->stream));
      if (ctx->tflags_cap < nf) {
        (void)dfree(ctx->d_tflags);
        ctx->d_tflags = nullptr;
        ctx->tflags_cap = 0;
        if (dalloc(&ctx->d_tflags, nf) != hipSuccess) return SR_ENOMEM;
        ctx->tflags_cap = nf;
      }
      if (ctx->skip_cap < ns) {
        (void)dfree(ctx->d_skip);
        ctx->d_skip = nullptr;
        ctx->skip_cap = 0;
        const int64_t c = std::max<int64_t>(4096, 2 * ns);
        if (dalloc(&ctx->d_skip, c) != hipSuccess) return SR_ENOMEM;
        ctx->skip_cap = c;
      }
    }
    HC(hipMemsetAsync(ctx->d_skip, 0, (size_t)ns * 4, ctx->stream));
  }
  const int64_t replays0 = ctx->graph_replays;
  auto flush = [&]() -> sr_status {
    if (q == 0) return SR_OK;
    if (ctx->bstore) {
      int64_t covered = 0;
      const sr_status rb = bs_flush(ctx, q, n_new, &covered);
      if (rb != SR_OK) return rb;
      pairs += covered * q;  // the pass updates these entries once per deferred block
      ++passes;
      q = 0;
      return SR_OK;
    }
    // the nodes the pass reaches: those with a nonzero panel row in one of its deferred
    // blocks; every other row and column of the pass's update is an exact zero
    const int64_t gstride = ctx->p_rows * ctx->pld;
    const int32_t words = (int32_t)((n_new + 31) / 32);
    int64_t* cnt_dev = ctx->d_act_cnt + passes;
    HC(hipMemsetAsync(ctx->d_act_bits, 0, (size_t)words * 4, ctx->stream));
    HC(launch_pass_rows(ctx->Pb, ctx->pld, gstride, q, 2 * (ctx->cfg.K + 1), n_new,
                        ctx->d_act_bits, ctx->stream));
    HC(launch_bits_to_list(ctx->d_act_bits, n_new, words, ctx->d_act, cnt_dev, ctx->stream));
    if (tskip)
      HC(launch_tile_flags(ctx->Pb, ctx->pld, gstride, q, ctx->d_act, cnt_dev, n_new,
                           ctx->d_tflags, tf_ld, ctx->d_skip + skip_blocks * steps_used,
                           steps_used, ctx->stream));
    LowRankArgs la{};
    la.S = ctx->S;
    la.P = ctx->Pb;
    la.pld = ctx->pld;
    la.gstride = gstride;
    la.p_rows = ctx->p_rows;
    la.r = q * ctx->pld;
    la.rows = nullptr;
    la.nrows = n_new;
    la.ncols = n_new;
    la.fused = 1;
    la.variant = ctx->gemm_variant;
    la.act = ctx->d_act;
    la.act_n = cnt_dev;
    if (tskip) {
      la.tflags = ctx->d_tflags;
      la.tf_ld = tf_ld;
      skip_blocks += q;
    }
    HC(run_lowrank(ctx, la));
    pass_blocks.push_back(q);
    ++passes;
    q = 0;
    return SR_OK;
  };

  // Incremental corrections (fused form, panel width 32 or 64): the blocks of a chunk that
  // read columns of S (low-rank and C1 blocks) take slots. When a deferred block has its
  // panel segment, it adds its terms to the correction vectors of the chunk's later slots
  // (launch_corr_update); a block then reads S[:, I] and S[:, j] as the stored columns plus
  // its two vectors, instead of correcting them from the whole deferred panel. The chunk
  // boundaries are the flushes: after `chunk` deferred blocks, or before a block that would
  // take more than corr_slots slots (C1 blocks between the deferred ones also take slots).
  const bool incremental = fused && (ctx->pld == 32 || ctx->pld == 64);
  if (incremental && !ctx->corr) {
    ctx->corr_slots = 2 * chunk + 32;
    if (dalloc(&ctx->corr, 2 * (int64_t)ctx->corr_slots * ctx->p_rows) != hipSuccess ||
        dalloc(&ctx->corr_w, 2 * (int64_t)ctx->corr_slots * 64) != hipSuccess)
      return SR_ENOMEM;
  }
  std::vector<int> slot_of(plan.size(), -1), chunk_of(plan.size(), 0);
  std::vector<char> flush_before(plan.size(), 0);
  std::vector<int> chunk_base{0};  // first slot of chunk c; chunk c ends at chunk_base[c + 1]
  std::vector<int32_t> rstart{0}, sinks, rows;
  if (incremental) {
    int cid = 0, nsl = 0, qp = 0, total = 0;
    for (size_t bi = 0; bi < plan.size(); ++bi) {
      const Block& b = plan[bi];
      const bool low = b.case_id == 0 || b.case_id == 2;
      const bool reads = low || b.case_id == 1;
      if (reads && nsl == ctx->corr_slots) {
        flush_before[bi] = 1;
        ++cid;
        chunk_base.push_back(total);
        nsl = qp = 0;
      }
      chunk_of[bi] = cid;
      if (reads) {
        slot_of[bi] = total++;
        ++nsl;
        if (b.case_id != 2) rows.insert(rows.end(), b.I.begin(), b.I.end());
        rstart.push_back((int32_t)rows.size());
        sinks.push_back(low ? b.j : -1);
      }
      if (low && ++qp == chunk) {
        ++cid;
        chunk_base.push_back(total);
        nsl = qp = 0;
      }
    }
    chunk_base.push_back(total);
    // slot table: rstart | sink | rows, uploaded once per batch (after the previous batch's
    // kernels, which read the old table, have run)
    std::vector<int32_t> tab(rstart);
    tab.insert(tab.end(), sinks.begin(), sinks.end());
    tab.insert(tab.end(), rows.begin(), rows.end());
    HC(hipStreamSynchronize(ctx->stream));
    if ((int64_t)tab.size() > ctx->corr_tab_cap) {
      (void)dfree(ctx->corr_tab);
      ctx->corr_tab = nullptr;
      ctx->corr_tab_cap = 0;
      const int64_t c = std::max<int64_t>(1024, 2 * (int64_t)tab.size());
      if (dmalloc((void**)&ctx->corr_tab, (size_t)c * 4) != hipSuccess) return SR_ENOMEM;
      ctx->corr_tab_cap = c;
    }
    HC(hipMemcpy(ctx->corr_tab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice));
  }
  const int nslots = (int)sinks.size();
  CorrSlots cs{};
  if (incremental) {
    cs.rstart = ctx->corr_tab;
    cs.sink = ctx->corr_tab + nslots + 1;
    cs.rows = ctx->corr_tab + 2 * nslots + 1;
    cs.corr = ctx->corr;
    cs.ldc = ctx->p_rows;
    cs.w = ctx->corr_w;
  }

  std::vector<const int32_t*> dev_of;
  r = stage_long_lists(ctx, plan, dev_of);
  if (r != SR_OK) return r;
  ctx->last_plan.clear();
  int cur_chunk = -1;
  for (size_t bi = 0; bi < plan.size(); ++bi) {
    const Block& b = plan[bi];
    bc[b.case_id]++;
    ctx->last_plan.push_back(b.case_id);
    ctx->last_plan.push_back(b.op);
    ctx->last_plan.push_back(b.j);
    ctx->last_plan.push_back((int32_t)b.dj);
    ctx->last_plan.push_back((int32_t)b.I.size());
    for (int32_t i : b.I) ctx->last_plan.push_back(i);
    if (incremental && flush_before[bi]) {
      r = flush();
      if (r != SR_OK) return r;
    }
    if (incremental && chunk_of[bi] != cur_chunk) {
      // a new chunk: its slots' vectors start at zero
      cur_chunk = chunk_of[bi];
      cs.base = chunk_base[cur_chunk];
      const int64_t nv = 2 * (int64_t)(chunk_base[cur_chunk + 1] - cs.base);
      if (nv > 0) HC(hipMemsetAsync(ctx->corr, 0, (size_t)(nv * cs.ldc * 8), ctx->stream));
    }
    FusedTarget ft{ctx->Pb, ctx->p_rows * ctx->pld, ctx->pld, q * ctx->pld};
    ft.incremental = incremental;
    if (incremental && slot_of[bi] >= 0) {
      ft.cI = ctx->corr + (int64_t)2 * (slot_of[bi] - cs.base) * cs.ldc;
      ft.cJ = ft.cI + cs.ldc;
    }
    switch (b.case_id) {
      case 0:
      case 2:
        r = lowrank_block(ctx, b.case_id, b.op, b.I, b.j, n_new, nullptr, fused ? &ft : nullptr,
                          dev_of[bi]);
        ++lowrank;
        if (!ctx->bstore && !fused) pairs += n_new * n_new;
        if (r == SR_OK && incremental) {
          // this block's terms for the chunk's later slots
          const int s0 = slot_of[bi] + 1, s1 = chunk_base[chunk_of[bi] + 1];
          if (s1 > s0)
            HC(launch_corr_update(ctx->Pb + (int64_t)q * ctx->p_rows * ctx->pld, ctx->pld, n_new,
                                  cs, s0, s1, ctx->stream));
        }
        if (r == SR_OK && fused && ++q == chunk) r = flush();
        break;
      case 1:
        r = c1_block(ctx, b.I, b.j, n_new, fused ? &ft : nullptr, dev_of[bi]);
        pairs += 2 * n_new + 1;
        break;
      default:
        r = c3_block(ctx, b.I, b.j);
        pairs += (int64_t)b.I.size() + 1;
        break;
    }
    if (r != SR_OK) return r;
  }
  r = flush();
  if (r != SR_OK) return r;
  ctx->last_r = 0;
  ctx->last_case = -1;
  if (stats) {
    HC(hipStreamSynchronize(ctx->stream));
    memset(stats, 0, sizeof(*stats));
    int64_t entries = 0, skipped = 0;
    if (!pass_blocks.empty()) {
      // each block of a dense fused pass updates the square of the pass's reached nodes
      std::vector<int64_t> cnts(pass_blocks.size());
      HC(hipMemcpy(cnts.data(), ctx->d_act_cnt, cnts.size() * 8, hipMemcpyDeviceToHost));
      for (size_t p = 0; p < cnts.size(); ++p) {
        pairs += (int64_t)pass_blocks[p] * cnts[p] * cnts[p];
        entries += (int64_t)pass_blocks[p] * (cnts[p] * (cnts[p] + 1) / 2);
      }
    }
    if (tskip && skip_blocks > 0) {
      // a k-step skipped on the tiles of u positions (rows and columns both among them) is
      // skipped on the u (u + 1) / 2 distinct entries of their triangle
      std::vector<int32_t> u((size_t)(skip_blocks * steps_used));
      HC(hipMemcpy(u.data(), ctx->d_skip, u.size() * 4, hipMemcpyDeviceToHost));
      for (int32_t x : u) skipped += (int64_t)x * (x + 1) / 2;
    }
    stats->edges_in = cnt;
    stats->edges_net = net_edges;
    stats->blocks = (int64_t)plan.size();
    for (int c = 0; c < 4; ++c) stats->blocks_case[c] = bc[c];
    stats->lowrank_blocks = lowrank;
    stats->n_after = n_new;
    stats->pairs = pairs;
    stats->fused_passes = passes;
    stats->series_replays = (int32_t)(ctx->graph_replays - replays0);
    stats->pass_entries = entries;
    stats->pass_skipped = skipped;
  }
  return SR_OK;
}

sr_status apply_batch_columns(sr_ctx* ctx, int64_t cnt, const int32_t* bi, const int32_t* bj,
                              const int8_t* bo, const int32_t* cols, int32_t ncols,
                              double* out_dev, int64_t ld_out, sr_batch_stats* stats) {
  if (!valid_ctx(ctx)) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  if (cnt < 0 || (cnt > 0 && (!bi || !bj || !bo)) || ncols < 0 ||
      (ncols > 0 && (!cols || !out_dev)))
    return SR_EINVAL;
  if (ctx->cfg.mode != SR_COLUMN || ctx->weighted) return SR_EMODE;
  const int64_t n = ctx->g.n;
  if (ld_out < n) return SR_EINVAL;
  for (int32_t t = 0; t < ncols; ++t)
    if (cols[t] < 0 || cols[t] >= n) return SR_ERANGE;
  std::vector<Block> plan;
  int64_t n_new = 0, net_edges = 0;
  sr_status r = plan_batch(ctx, cnt, bi, bj, bo, plan, n_new, net_edges);
  if (r != SR_OK) return r;
  if (n_new != n) return SR_EMODE;
  for (const Block& b : plan)
    if (b.case_id != 0) return SR_EMODE;

  hipStream_t s = ctx->stream;
  const double C = ctx->cfg.C;
  const int K = ctx->cfg.K;
  const int chunk = ctx->cfg.batch_chunk > 0 ? ctx->cfg.batch_chunk : 1;
  // Deferred blocks share one packed panel: block q's 2(K+1) columns are global columns
  // q 2(K+1) .. (q + 1) 2(K+1) - 1, stored in slabs of 16 columns (node-major inside a slab),
  // so the matrix-core pass runs over no padding but the last slab's tail. Rows past n stay
  // zero. The panel holds the slabs of `chunk` blocks, chunk 2(K+1) columns rounded up to 16.
  const int w = 2 * (K + 1);
  const int64_t slab = ctx->p_rows * 16;
  const int64_t slabs = ((int64_t)chunk * w + 15) / 16;
  auto at = [&](int64_t col) { return ctx->Pb + (col / 16) * slab + col % 16; };
  if (!ctx->Pb) {
    if (dalloc(&ctx->Pb, slabs * slab) != hipSuccess) return SR_ENOMEM;
    HC(hipMemsetAsync(ctx->Pb, 0, (size_t)(slabs * slab) * 8, s));
  }
  if (ncols > 0) {
    if (ctx->ids_cap < ncols) {
      HC(hipStreamSynchronize(s));
      (void)dfree(ctx->d_ids);
      ctx->d_ids = nullptr;
      ctx->ids_cap = 0;
      if (dalloc(&ctx->d_ids, ncols) != hipSuccess) return SR_ENOMEM;
      ctx->ids_cap = ncols;
    }
    HC(hipStreamSynchronize(s));
    HC(hipMemcpy(ctx->d_ids, cols, (size_t)ncols * 4, hipMemcpyHostToDevice));
    HC(hipMemsetAsync(out_dev, 0, (size_t)ncols * ld_out * 8, s));
  }
  int q = 0, passes = 0;
  auto flush = [&]() -> sr_status {
    if (q == 0 || ncols == 0) {
      q = 0;
      return SR_OK;
    }
    // columns past the last block in its slab may hold an earlier pass's values: clear them
    const int64_t rc = (int64_t)q * w;
    if (rc % 16)
      HC(hipMemset2DAsync(at(rc), 16 * 8, 0, (size_t)(16 - rc % 16) * 8, (size_t)ctx->p_rows,
                          s));
    LowRankArgs la{};
    la.P = ctx->Pb;
    la.pld = 16;
    la.gstride = slab;
    la.p_rows = ctx->p_rows;
    la.r = (int)((rc + 15) / 16 * 16);
    la.rows = ctx->d_ids;
    la.nrows = ncols;
    la.ncols = n;
    la.acc_out = out_dev;
    la.ld_out = ld_out;
    HC(profiled(ctx, [&]() { return launch_lowrank_acc(la, s); }));
    ++passes;
    q = 0;
    return SR_OK;
  };
  std::vector<const int32_t*> dev_of;
  r = stage_long_lists(ctx, plan, dev_of);
  if (r != SR_OK) return r;
  ctx->last_plan.clear();
  for (size_t bx = 0; bx < plan.size(); ++bx) {
    const Block& b = plan[bx];
    ctx->last_plan.push_back(b.case_id);
    ctx->last_plan.push_back(b.op);
    ctx->last_plan.push_back(b.j);
    ctx->last_plan.push_back((int32_t)b.dj);
    ctx->last_plan.push_back((int32_t)b.I.size());
    for (int32_t i : b.I) ctx->last_plan.push_back(i);
    const int64_t c0 = (int64_t)q * w;  // this block's first packed column
    // S[:, I] and S[:, j] on the current graph (PartialSim), Q S[:, I], then Table 2 (C0)
    const IdList il = idlist(b.I, 0, b.I.size(), dev_of[bx]);
    IdList lj;
    lj.count = 1;
    lj.id[0] = b.j;
    r = partial_sim2(ctx, il, lj, ctx->SI, ctx->Sj);
    if (r != SR_OK) return r;
    HC(launch_spmv_q(devq(ctx), heavy_args(ctx->hin), n, ctx->SI, ctx->QSI, 1.0, s));
    if (il.dev) HC(launch_sum_at(ctx->SI, il, ctx->d_sum, s));
    GammaArgs ga{};
    ga.kind = 0;
    ga.op = b.op;
    ga.j = b.j;
    ga.delta = (int32_t)b.I.size();
    ga.dj = ctx->g.in.len[b.j];
    ga.C = C;
    ga.xi0 = C;
    ga.I = il;
    ga.sumI = il.dev ? ctx->d_sum : nullptr;
    HC(launch_gamma(ga, n, ctx->SI, ctx->Sj, ctx->QSI, nullptr, nullptr, at(c0), 16, nullptr,
                    s));
    std::vector<std::pair<int32_t, int32_t>> e;
    for (int32_t i : b.I) e.push_back({i, b.j});
    r = edit_graph(ctx, e, b.op);
    if (r != SR_OK) return r;
    // step k reads (xi_k, eta_k): from the panel at k = 0, else from the compact copy the
    // previous step wrote; it writes (xi_{k+1}, eta_{k+1}) to the panel and a compact copy
    for (int k = 0; k < K; ++k) {
      const double* src = k == 0 ? at(c0) : ctx->pairs + ((k - 1) % 2) * 2 * ctx->node_cap;
      double* cdst = ctx->pairs + (k % 2) * 2 * ctx->node_cap;
      HC(launch_series_step_to(devq(ctx), heavy_args(ctx->hin), n, at(c0 + 2 * (k + 1)), 16,
                               src, k == 0 ? 16 : 2, cdst, C, 1.0, s));
    }
    if (++q == chunk) {
      r = flush();
      if (r != SR_OK) return r;
    }
  }
  r = flush();
  if (r != SR_OK) return r;
  ctx->last_r = 0;  // the single-update series state no longer describes the graph
  ctx->last_case = -1;
  if (stats) {
    HC(hipStreamSynchronize(s));
    memset(stats, 0, sizeof(*stats));
    stats->edges_in = cnt;
    stats->edges_net = net_edges;
    stats->blocks = (int64_t)plan.size();
    stats->blocks_case[0] = (int64_t)plan.size();
    stats->lowrank_blocks = (int64_t)plan.size();
    stats->n_after = n;
    stats->pairs = (int64_t)plan.size() * n * ncols;
    stats->fused_passes = passes;
  }
  return SR_OK;
}

sr_status sr_last_plan(sr_ctx* ctx, int32_t* out, int64_t cap, int64_t* len) {
  if (!valid_ctx(ctx) || !len) return SR_EINVAL;
  *len = (int64_t)ctx->last_plan.size();
  if (out && cap >= *len) memcpy(out, ctx->last_plan.data(), ctx->last_plan.size() * 4);
  return SR_OK;
}

// ------------------------------------------------------------------------------ queries

// Delta S columns of the last unit update (eq (71) for the low-rank cases C0 and C2; the new
// sink's column for C1; the new diagonals for C3): the list rows (device, ncols) or the single
// column x, as float32 (out32) or float64 (out64) rows of ld values.
static sr_status delta_columns(sr_ctx* ctx, const int32_t* rows, int32_t x, int32_t ncols,
                               float* out32, double* out64, int64_t ld) {
  const int64_t n = ctx->g.n;
  hipStream_t s = ctx->stream;
  const int c = ctx->last_case;
  if (c < 0) return SR_EMODE;
  if (c == 0 || c == 2) {
    if (ctx->last_r == 0) return SR_EMODE;
    if (out64) {
      HC(launch_delta_col(ctx->P, ctx->pld, ctx->last_r, n, x, out64, s));
    } else {
      LowRankArgs la{};
      la.P = ctx->P;
      la.pld = ctx->pld;
      la.gstride = ctx->p_rows * ctx->pld;
      la.p_rows = ctx->p_rows;
      la.r = ctx->last_r;
      la.rows = rows;
      la.nrows = ncols;
      la.ncols = n;
      la.out = out32;
      la.ld_out = ld;
      HC(run_lowrank(ctx, la));
    }
    if (c == 2)  // the new source's own column
      HC(launch_node_cols(rows, x, ncols, n, 2, ctx->last_i, ctx->last_j, nullptr, ctx->last_vi,
                          0.0, out32, out64, ld, s));
    return SR_OK;
  }
  HC(launch_node_cols(rows, x, ncols, n, c, ctx->last_i, ctx->last_j, ctx->ylast, ctx->last_vi,
                      ctx->last_vj, out32, out64, ld, s));
  return SR_OK;
}

sr_status query_column(sr_ctx* ctx, int32_t x, int32_t what, double* out_dev) {
  if (!valid_ctx(ctx) || !out_dev) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  const int64_t n = ctx->g.n;
  if (x < 0 || x >= n) return SR_ERANGE;
  if (what == SR_COL_S) {
    if (ctx->cfg.mode != SR_DENSE) return SR_EMODE;
    if (ctx->bstore) {
      const sr_status r = stage_ids(ctx, &x, 1);
      if (r != SR_OK) return r;
      HC(launch_bs_rows(bs_view(ctx), n, ctx->d_ids, 1, out_dev, nullptr, n, ctx->stream));
      return SR_OK;
    }
    HC(launch_copy_row(ctx->S, n, x, out_dev, ctx->stream));
    return SR_OK;
  }
  if (what != SR_COL_DELTA) return SR_EINVAL;
  return delta_columns(ctx, nullptr, x, 1, nullptr, out_dev, n);
}

sr_status query_columns(sr_ctx* ctx, const int32_t* cols, int32_t ncols, float* out_dev,
                        int64_t ld_out) {
  if (!valid_ctx(ctx) || !cols || !out_dev || ncols < 0) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  const int64_t n = ctx->g.n;
  if (ld_out < n) return SR_EINVAL;
  for (int32_t t = 0; t < ncols; ++t)
    if (cols[t] < 0 || cols[t] >= n) return SR_ERANGE;
  if (ncols == 0) return SR_OK;
  if (ctx->ids_cap < ncols) {
    HC(hipStreamSynchronize(ctx->stream));
    (void)dfree(ctx->d_ids);
    ctx->d_ids = nullptr;
    ctx->ids_cap = 0;
    if (dalloc(&ctx->d_ids, ncols) != hipSuccess) return SR_ENOMEM;
    ctx->ids_cap = ncols;
  }
  HC(hipStreamSynchronize(ctx->stream));  // d_ids may be read by earlier work
  HC(hipMemcpy(ctx->d_ids, cols, (size_t)ncols * 4, hipMemcpyHostToDevice));
  if (ctx->cfg.mode == SR_DENSE && ctx->bstore) {
    HC(launch_bs_rows(bs_view(ctx), n, ctx->d_ids, ncols, nullptr, out_dev, ld_out,
                      ctx->stream));
    return SR_OK;
  }
  if (ctx->cfg.mode == SR_DENSE) {
    HC(launch_rows_to_f32(ctx->S, n, ctx->d_ids, ncols, out_dev, ld_out, ctx->stream));
    return SR_OK;
  }
  return delta_columns(ctx, ctx->d_ids, -1, ncols, out_dev, nullptr, ld_out);
}

sr_status query_topk(sr_ctx* ctx, const int32_t* q, int32_t nq, int32_t k,
                     int32_t exclude_self, int32_t* idx_dev, double* val_dev) {
  if (!valid_ctx(ctx) || nq < 0 || (nq > 0 && (!q || !idx_dev || !val_dev))) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  const int64_t n = ctx->g.n;
  if (k < 1 || k > kTopkMax || k > n - (exclude_self ? 1 : 0)) return SR_EINVAL;
  for (int32_t t = 0; t < nq; ++t)
    if (q[t] < 0 || q[t] >= n) return SR_ERANGE;
  if (nq == 0) return SR_OK;
  if (ctx->ids_cap < nq) {
    HC(hipStreamSynchronize(ctx->stream));
    (void)dfree(ctx->d_ids);
    ctx->d_ids = nullptr;
    ctx->ids_cap = 0;
    if (dalloc(&ctx->d_ids, nq) != hipSuccess) return SR_ENOMEM;
    ctx->ids_cap = nq;
  }
  HC(hipStreamSynchronize(ctx->stream));  // d_ids may be read by earlier work
  HC(hipMemcpy(ctx->d_ids, q, (size_t)nq * 4, hipMemcpyHostToDevice));
  hipStream_t s = ctx->stream;
  const int ex = exclude_self ? 1 : 0;
  if (ctx->cfg.mode == SR_DENSE && ctx->bstore) {
    // the queries' rows of S gathered from the block pairs, then selected as vectors
    const int64_t chunk = std::min<int64_t>(nq, kStoreTopkRows);
    double* rows = nullptr;
    if (dalloc(&rows, chunk * n) != hipSuccess) return SR_ENOMEM;
    hipError_t e = hipSuccess;
    for (int64_t t = 0; t < nq && e == hipSuccess; t += chunk) {
      const int c = (int)std::min<int64_t>(chunk, nq - t);
      e = launch_bs_rows(bs_view(ctx), n, ctx->d_ids + t, c, rows, nullptr, n, s);
      if (e == hipSuccess)
        e = profiled(ctx, [&]() {
          return launch_topk(ctx->S, rows, n, ctx->d_ids + t, c, n, k, ex, idx_dev + t * k,
                             val_dev + t * k, s);
        });
    }
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)dfree(rows);
    HC(e);
    HC(e2);
    return SR_OK;
  }
  if (ctx->cfg.mode == SR_DENSE) {
    HC(profiled(ctx, [&]() {
      return launch_topk(ctx->S, nullptr, 0, ctx->d_ids, nq, n, k, ex, idx_dev, val_dev, s);
    }));
    return SR_OK;
  }
  // column mode: the PartialSim columns of two queries at a time, then their selections
  for (int32_t t = 0; t < nq; t += 2) {
    IdList a, b;
    a.count = b.count = 1;
    a.id[0] = q[t];
    b.id[0] = q[t + 1 < nq ? t + 1 : t];
    sr_status r = partial_sim2(ctx, a, b, ctx->SI, ctx->Sj);
    if (r != SR_OK) return r;
    HC(profiled(ctx, [&]() {
      return launch_topk(ctx->S, ctx->SI, 0, ctx->d_ids + t, 1, n, k, ex,
                         idx_dev + (int64_t)t * k, val_dev + (int64_t)t * k, s);
    }));
    if (t + 1 < nq)
      HC(profiled(ctx, [&]() {
        return launch_topk(ctx->S, ctx->Sj, 0, ctx->d_ids + t + 1, 1, n, k, ex,
                           idx_dev + (int64_t)(t + 1) * k, val_dev + (int64_t)(t + 1) * k, s);
      }));
  }
  return SR_OK;
}

sr_status query_topk_noalloc(sr_ctx* ctx, const int32_t* q, int32_t nq, int32_t k,
                             int32_t exclude_self, int32_t* idx_dev, double* val_dev) {
  if (!valid_ctx(ctx) || nq < 0 || (nq > 0 && (!q || !idx_dev || !val_dev))) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  const int64_t n = ctx->g.n;
  if (k < 1 || k > kTopkMax || k > n - (exclude_self ? 1 : 0)) return SR_EINVAL;
  if (nq > kScratchIds) return SR_ECAPACITY;
  if (ctx->bstore) return SR_EMODE;  // the block store's selection stages rows
  for (int32_t t = 0; t < nq; ++t)
    if (q[t] < 0 || q[t] >= n) return SR_ERANGE;
  if (nq == 0) return SR_OK;
  int32_t* ids = (ctx->device >= 0 && ctx->device < kMaxDevices) ? scratch_ptr[ctx->device]
                                                                 : nullptr;
  if (!ids) return SR_EHIP;
  hipStream_t s = ctx->stream;
  const int ex = exclude_self ? 1 : 0;
  // stream-ordered: an earlier call's kernels on this stream have read the previous ids
  HC(hipMemcpyAsync(ids, q, (size_t)nq * 4, hipMemcpyHostToDevice, s));
  if (ctx->cfg.mode == SR_DENSE) {
    HC(launch_topk(ctx->S, nullptr, 0, ids, nq, n, k, ex, idx_dev, val_dev, s));
    return SR_OK;
  }
  for (int32_t t = 0; t < nq; t += 2) {
    IdList a, b;
    a.count = b.count = 1;
    a.id[0] = q[t];
    b.id[0] = q[t + 1 < nq ? t + 1 : t];
    sr_status r = partial_sim2(ctx, a, b, ctx->SI, ctx->Sj);
    if (r != SR_OK) return r;
    HC(launch_topk(ctx->S, ctx->SI, 0, ids + t, 1, n, k, ex, idx_dev + (int64_t)t * k,
                   val_dev + (int64_t)t * k, s));
    if (t + 1 < nq)
      HC(launch_topk(ctx->S, ctx->Sj, 0, ids + t + 1, 1, n, k, ex,
                     idx_dev + (int64_t)(t + 1) * k, val_dev + (int64_t)(t + 1) * k, s));
  }
  return SR_OK;
}

sr_status sr_gather_pairs(sr_ctx* ctx, int64_t np, const int32_t* a, const int32_t* b,
                          double* out) {
  if (!valid_ctx(ctx) || np < 0 || (np > 0 && (!a || !b || !out))) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  if (ctx->cfg.mode != SR_DENSE) return SR_EMODE;
  const sr_status rs = check_pair_ids(ctx, np, a, b);
  if (rs != SR_OK) return rs;
  if (ctx->bstore) {
    HC(launch_bs_pairs(bs_view(ctx), np, a, b, out, ctx->stream));
    return SR_OK;
  }
  HC(launch_gather_pairs(ctx->S, np, a, b, out, ctx->stream));
  return SR_OK;
}

sr_status sr_copy_S(sr_ctx* ctx, double* out_dev, int64_t ld) {
  if (!valid_ctx(ctx) || !out_dev) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  if (ctx->cfg.mode != SR_DENSE) return SR_EMODE;
  if (ld < ctx->g.n) return SR_EINVAL;
  if (ctx->bstore) {
    const int64_t n = ctx->g.n;
    std::vector<int32_t> all(n);
    for (int64_t v = 0; v < n; ++v) all[v] = (int32_t)v;
    const sr_status r = stage_ids(ctx, all.data(), n);
    if (r != SR_OK) return r;
    HC(launch_bs_rows(bs_view(ctx), n, ctx->d_ids, n, out_dev, nullptr, ld, ctx->stream));
    return SR_OK;
  }
  HC(launch_from_store(ctx->S, ctx->g.n, out_dev, ld, ctx->stream));
  return SR_OK;
}

sr_status sr_get_aff(sr_ctx* ctx, int32_t level, int32_t* A_dev, int64_t* nA, int32_t* B_dev,
                     int64_t* nB) {
  if (!valid_ctx(ctx) || !nA || !nB) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  if (!ctx->last_aff) return SR_EMODE;
  if (level < -1 || level > ctx->cfg.K) return SR_ERANGE;
  const uint32_t* a = level < 0 ? ctx->Ahat : ctx->Abits + (int64_t)level * ctx->W;
  const uint32_t* b = level < 0 ? ctx->Bhat : ctx->Bbits + (int64_t)level * ctx->W;
  HC(launch_bits_to_list(a, ctx->g.n, ctx->W, A_dev, ctx->d_cnt + 4, ctx->stream));
  HC(launch_bits_to_list(b, ctx->g.n, ctx->W, B_dev, ctx->d_cnt + 5, ctx->stream));
  HC(hipMemcpyAsync(ctx->h_cnt + 4, ctx->d_cnt + 4, 2 * sizeof(int64_t), hipMemcpyDeviceToHost,
                    ctx->stream));
  HC(hipStreamSynchronize(ctx->stream));
  *nA = ctx->h_cnt[4];
  *nB = ctx->h_cnt[5];
  return SR_OK;
}

sr_status sr_edges(sr_ctx* ctx, int32_t* src, int32_t* dst, double* w, int64_t cap,
                   int64_t* m) {
  if (!valid_ctx(ctx) || !m) return SR_EINVAL;
  *m = ctx->g.m;
  if (cap < *m) return SR_OK;  // size query
  if (!ctx->updated) {
    for (int64_t e = 0; e < *m; ++e) {
      if (src) src[e] = ctx->src0[e];
      if (dst) dst[e] = ctx->dst0[e];
      if (w) w[e] = ctx->weighted ? ctx->w0[e] : 1.0;
    }
    return SR_OK;
  }
  const SlotList& L = ctx->g.in;
  int64_t k = 0;
  for (int64_t j = 0; j < ctx->g.n; ++j)
    for (int32_t p = 0; p < L.len[j]; ++p, ++k) {
      const int64_t slot = L.start[j] + p;
      if (src) src[k] = L.idx[slot];
      if (dst) dst[k] = (int32_t)j;
      if (w) w[k] = ctx->weighted ? L.w[slot] : 1.0;
    }
  return SR_OK;
}

sr_status sr_sizes(sr_ctx* ctx, int64_t* n, int64_t* m) {
  if (!valid_ctx(ctx)) return SR_EINVAL;
  if (n) *n = ctx->g.n;
  if (m) *m = ctx->g.m;
  return SR_OK;
}

sr_status sr_get_config(sr_ctx* ctx, sr_config* out) {
  if (!valid_ctx(ctx) || !out) return SR_EINVAL;
  *out = ctx->cfg;
  return SR_OK;
}

sr_status sr_store_bytes(sr_ctx* ctx, int64_t* bytes, int64_t* pairs) {
  if (!valid_ctx(ctx)) return SR_EINVAL;
  int64_t b = 0, np = 0;
  if (ctx->bstore) {
    b = ctx->bs_bytes;
    for (const SView& v : ctx->bs_pairs) np += v.d != nullptr;
  } else if (ctx->cfg.mode == SR_DENSE) {
    b = ctx->node_cap * ctx->S.ld * (ctx->cfg.s_prec == SR_S_FP32 ? 4 : 8);
  }
  if (bytes) *bytes = b;
  if (pairs) *pairs = np;
  return SR_OK;
}

sr_status sr_device_bytes(int64_t* held, int64_t* peak, int32_t reset_peak) {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  if (held) *held = g_mem_now;
  if (peak) *peak = g_mem_peak;
  if (reset_peak) g_mem_peak = g_mem_now;
  return SR_OK;
}

sr_status sr_synchronize(sr_ctx* ctx) {
  if (!valid_ctx(ctx)) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  HC(hipStreamSynchronize(ctx->stream));
  return SR_OK;
}

// ------------------------------------------------------------------------------ adjoint

sr_status backward(sr_ctx* ctx, int64_t npairs, const int32_t* a_dev, const int32_t* b_dev,
                   const double* g_dev, double* dw_dev) {
  if (!valid_ctx(ctx) || npairs < 0 || !dw_dev || (npairs > 0 && (!a_dev || !b_dev || !g_dev)))
    return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  if (ctx->cfg.mode != SR_DENSE || ctx->bstore) return SR_EMODE;
  {
    const sr_status rs = check_pair_ids(ctx, npairs, a_dev, b_dev);
    if (rs != SR_OK) return rs;
  }
  const int64_t n = ctx->g.n;
  const int64_t m = ctx->g.m;
  const double C = ctx->cfg.C;
  hipStream_t s = ctx->stream;
  const int64_t ldi = (n + 63) / 64 * 64;
  double *Sig = nullptr, *T = nullptr, *U = nullptr, *G = nullptr, *dq = nullptr, *qv = nullptr;
  int32_t* se = nullptr;
  auto cleanup = [&]() {
    (void)dfree(Sig);
    (void)dfree(T);
    (void)dfree(U);
    (void)dfree(G);
    (void)dfree(dq);
    (void)dfree(qv);
    (void)dfree(se);
  };
  if (dalloc(&Sig, n * ldi) != hipSuccess || dalloc(&T, n * ldi) != hipSuccess ||
      dalloc(&U, n * ldi) != hipSuccess || dalloc(&G, n * ldi) != hipSuccess ||
      dalloc(&dq, (int64_t)ctx->g.in.idx.size()) != hipSuccess ||
      dalloc(&qv, (int64_t)ctx->g.out.idx.size()) != hipSuccess ||
      dalloc(&se, (int64_t)ctx->slot_edge0.size()) != hipSuccess) {
    cleanup();
    return SR_ENOMEM;
  }
  const DevQ q = devq(ctx);
  const DevAdj out = devout(ctx);
  // in-list slot -> output position: the caller's edge order until the first update, then
  // the order of sr_edges (sinks ascending, slots in order)
  const std::vector<int32_t> se_host = ctx->updated ? slot_edges(ctx) : ctx->slot_edge0;
  hipError_t e = hipMemcpy(se, se_host.data(), se_host.size() * 4, hipMemcpyHostToDevice);
  // Gs = G + G^T: Sig = Lam + Lam^T solves Sig = Gs + C Q^T Sig Q (Lam = G + C Q^T Lam Q).
  if (e == hipSuccess) e = launch_qt_values(q, out, n, qv, s);
  if (e == hipSuccess) e = hipMemsetAsync(G, 0, (size_t)n * ldi * 8, s);
  if (e == hipSuccess) e = launch_scatter_pairs_sym(G, n, npairs, a_dev, b_dev, g_dev, s);
  if (e == hipSuccess) e = hipMemcpyAsync(Sig, G, (size_t)n * ldi * 8,
                                          hipMemcpyDeviceToDevice, s);
  // Sig symmetric: Q^T Sig Q = Q^T (Q^T Sig)^T, so U = Q^T Sig, T = U^T, Sig' = Gs + C Q^T T.
  for (int it = 0; it < ctx->cfg.init_max_iter && e == hipSuccess; ++it) {
    e = hipMemsetAsync(ctx->d_max, 0, 8, s);
    if (e == hipSuccess) e = profiled(ctx, [&]() {
      return launch_spmm_qt_rows(out, qv, n, Sig, U, 1.0, nullptr, nullptr, nullptr, s);
    });
    if (e == hipSuccess) e = launch_transpose(n, U, T, s);
    if (e == hipSuccess) e = profiled(ctx, [&]() {
      return launch_spmm_qt_rows(out, qv, n, T, U, C, G, Sig, ctx->d_max, s);
    });
    if (e == hipSuccess) e = hipMemcpyAsync(ctx->h_max, ctx->d_max, 8, hipMemcpyDeviceToHost,
                                            s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    std::swap(Sig, U);
    double step;
    memcpy(&step, ctx->h_max, 8);
    if (step <= ctx->cfg.init_tol) break;
  }
  // T = (Q S)^T: T = S (float64), U = Q T, T = U^T.
  if (e == hipSuccess) e = launch_from_store(ctx->S, n, T, ldi, s);
  if (e == hipSuccess) e = launch_spmm_rows(q, n, T, U, 1.0, 0.0, nullptr, nullptr, s);
  if (e == hipSuccess) e = launch_transpose(n, U, T, s);
  if (e == hipSuccess) e = launch_edge_grad(q, n, Sig, T, C, se, dq, dw_dev, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
  (void)m;
  if (e != hipSuccess) return fail_hip(ctx);
  return SR_OK;
}

sr_status sr_profile(sr_ctx* ctx, int32_t enable) {
  if (!valid_ctx(ctx)) return SR_EINVAL;
  ctx->profiling = enable != 0;
  return SR_OK;
}

sr_status sr_profile_read(sr_ctx* ctx, double* ms, int64_t* launches, int32_t reset) {
  if (!valid_ctx(ctx) || !ms || !launches) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  HC(hipStreamSynchronize(ctx->stream));
  for (auto& ev : ctx->prof_events) {
    float t = 0.0f;
    HC(hipEventElapsedTime(&t, ev.first, ev.second));
    ctx->prof_ms += t;
    ctx->prof_launches++;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  ctx->prof_events.clear();
  *ms = ctx->prof_ms;
  *launches = ctx->prof_launches;
  if (reset) {
    ctx->prof_ms = 0.0;
    ctx->prof_launches = 0;
  }
  return SR_OK;
}

sr_status sr_time_fused(sr_ctx* ctx, int32_t variant, int32_t blocks, int32_t reps,
                        double* gemm_ms, double* corr_ms) {
  if (!valid_ctx(ctx) || !gemm_ms || !corr_ms || blocks < 1 || reps < 1) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  if (ctx->cfg.mode != SR_DENSE || ctx->bstore) return SR_EMODE;
  if (variant < 0 || variant >= kGemmVariants) return SR_ERANGE;
  const int64_t n = ctx->g.n;
  const int pld = ctx->pld;
  const int64_t cols = (int64_t)blocks * pld;
  hipStream_t s = ctx->stream;
  double* Z = nullptr;  // a zero panel: the timed passes add exact zeros to S
  int32_t* tab = nullptr;
  int32_t* act = nullptr;  // every node listed: the passes' reached-node code path
  int64_t* act_n = nullptr;
  double *cv = nullptr, *cw = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int slots = std::max(1, blocks / 2);
  auto done = [&](sr_status r) {
    (void)hipStreamSynchronize(s);
    (void)dfree(Z);
    (void)dfree(tab);
    (void)dfree(act);
    (void)dfree(act_n);
    (void)dfree(cv);
    (void)dfree(cw);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return r;
  };
  if (dalloc(&Z, ctx->p_rows * cols) != hipSuccess || dalloc(&tab, 2 * slots + 1) != hipSuccess ||
      dalloc(&cv, 2 * (int64_t)slots * ctx->p_rows) != hipSuccess ||
      dalloc(&cw, 2 * (int64_t)slots * pld) != hipSuccess || dalloc(&act, n) != hipSuccess ||
      dalloc(&act_n, 1) != hipSuccess)
    return done(SR_ENOMEM);
  {
    std::vector<int32_t> ids(n);
    for (int64_t a = 0; a < n; ++a) ids[a] = (int32_t)a;
    const int64_t cnt = n;
    if (hipMemcpy(act, ids.data(), (size_t)n * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(act_n, &cnt, 8, hipMemcpyHostToDevice) != hipSuccess) {
      ctx->poisoned = true;
      return done(SR_EHIP);
    }
  }
  if (hipMemsetAsync(Z, 0, (size_t)ctx->p_rows * cols * 8, s) != hipSuccess ||
      hipMemsetAsync(tab, 0, (size_t)(2 * slots + 1) * 4, s) != hipSuccess ||
      hipMemsetAsync(cv, 0, (size_t)2 * slots * ctx->p_rows * 8, s) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    ctx->poisoned = true;
    return done(SR_EHIP);
  }
  LowRankArgs la{};
  la.S = ctx->S;
  la.P = Z;
  la.pld = pld;
  la.gstride = ctx->p_rows * pld;
  la.p_rows = ctx->p_rows;
  la.r = (int)cols;
  la.nrows = n;
  la.ncols = n;
  la.fused = 1;
  la.variant = variant;
  la.act = act;
  la.act_n = act_n;
  // one deferred block's corrections for `slots` later slots of its chunk (zero weights)
  CorrSlots cs{};
  cs.rstart = tab;
  cs.sink = tab + slots + 1;
  cs.rows = tab;
  cs.corr = cv;
  cs.ldc = ctx->p_rows;
  cs.base = 0;
  cs.w = cw;
  float t_gemm = 0.0f, t_corr = 0.0f;
  hipError_t e = launch_lowrank(la, s);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_lowrank(la, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&t_gemm, e0, e1);
  if (e == hipSuccess && (pld == 32 || pld == 64)) {
    e = launch_corr_update(Z, pld, n, cs, 0, slots, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_corr_update(Z, pld, n, cs, 0, slots, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t_corr, e0, e1);
  }
  if (e != hipSuccess) {
    ctx->poisoned = true;
    return done(SR_EHIP);
  }
  *gemm_ms = (double)t_gemm / reps;
  *corr_ms = (double)t_corr / reps;
  return done(SR_OK);
}

sr_status sr_set_tuning(sr_ctx* ctx, int32_t batch_chunk, int32_t variant) {
  if (!valid_ctx(ctx) || batch_chunk < 1 || batch_chunk > kMaxChunk) return SR_EINVAL;
  if (ctx->poisoned) return SR_EHIP;
  if (variant < 0 || variant >= kGemmVariants) return SR_ERANGE;
  if (batch_chunk != ctx->cfg.batch_chunk) {
    // the batch panel and the correction slots are sized by the chunk: allocated again by
    // the next batch (captured chains keep panel addresses, so they go too)
    HC(hipStreamSynchronize(ctx->stream));
    for (auto& g : ctx->sgraphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    ctx->sgraphs.clear();
    double* bufs[] = {ctx->Pb, ctx->wts, ctx->corr, ctx->corr_w};
    for (double* b : bufs) (void)dfree(b);
    ctx->Pb = ctx->wts = ctx->corr = ctx->corr_w = nullptr;
    ctx->corr_slots = 0;
    ctx->cfg.batch_chunk = batch_chunk;
  }
  ctx->gemm_variant = variant;
  return SR_OK;
}

sr_status sr_mfma_layout_probe_f32(const float* a_dev, const float* b_dev, float* out_dev,
                                   void* hip_stream) {
  if (!a_dev || !b_dev || !out_dev) return SR_EINVAL;
  return launch_mfma_probe_f32(a_dev, b_dev, out_dev, (hipStream_t)hip_stream) == hipSuccess
             ? SR_OK
             : SR_EHIP;
}

sr_status sr_mfma_layout_probe(const double* a_dev, const double* b_dev, double* out_dev,
                               void* hip_stream) {
  if (!a_dev || !b_dev || !out_dev) return SR_EINVAL;
  return launch_mfma_probe(a_dev, b_dev, out_dev, (hipStream_t)hip_stream) == hipSuccess
             ? SR_OK
             : SR_EHIP;
}

}  // extern "C"
