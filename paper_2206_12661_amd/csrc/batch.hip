// Batched form: several independent plans iterated together.
//
// Every stage of a pass (forward product with the fused focus gather, focus
// update, scatter, adjoint product with the projection) is ONE grouped launch
// over all plans of the batch: the launch's workgroups are the concatenated
// tile lists of the plans' products, each workgroup finding its plan by a
// binary search over the item start offsets.  A pass of the whole batch is
// thus four launches whatever the number of plans, and it is replayed from a
// captured HIP graph.  The plans share one precision: float32 products with
// autotuned tiles, or the split-precision products with the single-plan
// form's loops.  Items are ordered by descending K (the longest tiles
// are dispatched first) so that the short products of small holograms fill
// the tail of the launch.
//
// Each plan's own arithmetic is exactly that of its single-plan pass with no
// K split: tiles, k order, reductions and epilogues are the same code, so a
// batched result equals the single-plan result bit for bit whenever the tiles
// are the same.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "gswmtp_internal.h"

using namespace gswmtp;

struct gswmtp_batch {
  int device = 0;
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_user = nullptr, ev_done = nullptr;
  std::vector<gswmtp_plan *> plans;
  std::vector<hipEvent_t> ev_plan;
  GroupedLaunch fwd, bwd;
  GroupedUpdate upd;
  void *d_sc = nullptr;
  int *d_sc_starts = nullptr;
  int sc_blocks = 0;
  int **d_ctrl = nullptr;
  double **d_stats = nullptr;
  void *pool = nullptr;
  hipGraphExec_t graph1 = nullptr, graph8 = nullptr;
  bool use_graph = true;
  double tune_ms[2][4] = {};   // [forward/adjoint][candidate] mean launch ms (0: not timed)
  int precision = GSWMTP_FP32; // common precision of the plans
  std::string err;
};

namespace {

thread_local std::string g_batch_create_error;

int bfail(gswmtp_batch *b, int code, const char *what, hipError_t e = hipSuccess) {
  if (b) {
    char buf[512];
    if (e != hipSuccess)
      snprintf(buf, sizeof buf, "%s: %s (%s)", what, hipGetErrorString(e), hipGetErrorName(e));
    else
      snprintf(buf, sizeof buf, "%s", what);
    b->err = buf;
  }
  return code;
}

#define BHIP_TRY(b, expr)                                        \
  do {                                                           \
    hipError_t e_ = (expr);                                      \
    if (e_ != hipSuccess) return bfail((b), GSWMTP_E_HIP, #expr, e_); \
  } while (0)

struct DeviceGuardB {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuardB(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuardB() {
    if (changed) (void)hipSetDevice(prev);
  }
};

// Run control of every plan (graph-safe: a kernel, not a memset).
__global__ void k_batch_control(int *const *ctrl, double *const *stats, int n, double stop) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ctrl[i][CTRL_DONE] = 0;
  ctrl[i][CTRL_NONFINITE] = 0;
  stats[i][ST_STOP] = stop;
}

constexpr int kCand[4][2] = {{64, 64}, {64, 128}, {128, 64}, {128, 128}};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

hipError_t enqueue_batch_pass(gswmtp_batch *b, hipStream_t s) {
  hipError_t e;
  const int n = (int)b->plans.size();
  if (b->precision != GSWMTP_FP32) {
    if ((e = launch_cgemm_split_grouped(b->fwd, s)) != hipSuccess) return e;
    if ((e = launch_update_grouped(b->upd, s)) != hipSuccess) return e;
    if ((e = launch_scatter_split_grouped(b->d_sc, b->d_sc_starts, n, b->sc_blocks, b->precision,
                                          s)) != hipSuccess)
      return e;
    return launch_cgemm_split_grouped(b->bwd, s);
  }
  if ((e = launch_cgemm_grouped(b->fwd, s)) != hipSuccess) return e;
  if ((e = launch_update_grouped(b->upd, s)) != hipSuccess) return e;
  if ((e = launch_scatter_grouped(b->d_sc, b->d_sc_starts, n, b->sc_blocks, s)) != hipSuccess)
    return e;
  return launch_cgemm_grouped(b->bwd, s);
}

hipError_t capture_batch(gswmtp_batch *b, int passes, hipGraphExec_t *out) {
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t le = hipSuccess;
  for (int i = 0; i < passes && le == hipSuccess; ++i) le = enqueue_batch_pass(b, b->stream);
  e = hipStreamEndCapture(b->stream, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return le;
  }
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

void free_batch(gswmtp_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->graph1) (void)hipGraphExecDestroy(b->graph1);
  if (b->graph8) (void)hipGraphExecDestroy(b->graph8);
  if (b->pool) (void)hipFree(b->pool);
  for (auto e : b->ev_plan)
    if (e) (void)hipEventDestroy(e);
  if (b->ev_user) (void)hipEventDestroy(b->ev_user);
  if (b->ev_done) (void)hipEventDestroy(b->ev_done);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

// Host image of one grouped product: items in dispatch order and their
// first-block offsets.
struct GroupedHost {
  std::vector<unsigned char> items;
  std::vector<int> starts;
  int blocks = 0;
};

// tuning: a timing run (no done flag; the adjoint's projected field goes to
// `scratch`, which holds 2 Rp Cp floats per plan, so no plan state changes).
GroupedHost build_grouped(const std::vector<gswmtp_plan *> &plans, const std::vector<int> &order,
                          bool forward, int bm, int bn, bool tuning, float *scratch) {
  const size_t sz = cgemm_args_bytes();
  GroupedHost g;
  g.items.resize(sz * order.size());
  g.starts.resize(order.size() + 1);
  size_t off = 0;
  for (size_t k = 0; k < order.size(); ++k) {
    const gswmtp_plan *p = plans[order[k]];
    float *cr = nullptr, *ci = nullptr;
    if (tuning && !forward) {
      const size_t n = (size_t)p->d.Rp * p->d.Cp;
      cr = scratch + off;
      ci = scratch + off + n;
      off += 2 * n;
    }
    g.starts[k] = g.blocks;
    g.blocks += fill_cgemm_args(p, forward, bm, bn, !tuning, cr, ci, g.items.data() + k * sz);
  }
  g.starts[order.size()] = g.blocks;
  return g;
}

bool tile_valid(const std::vector<gswmtp_plan *> &plans, bool forward, int bm, int bn) {
  for (const auto *p : plans) {
    const int M = forward ? p->d.Urp : p->d.Rp;
    if (M % bm || p->d.Cp % bn) return false;
  }
  return true;
}

// Device copies of a grouped product (items + starts) carved from `base`.
int upload_grouped(gswmtp_batch *b, const GroupedHost &h, char *&base, GroupedLaunch &g) {
  const size_t isz = align256(h.items.size()), ssz = align256(h.starts.size() * sizeof(int));
  g.d_items = base;
  g.d_starts = reinterpret_cast<int *>(base + isz);
  base += isz + ssz;
  g.n_items = (int)h.starts.size() - 1;
  g.blocks = h.blocks;
  BHIP_TRY(b, hipMemcpy(g.d_items, h.items.data(), h.items.size(), hipMemcpyHostToDevice));
  BHIP_TRY(b, hipMemcpy(g.d_starts, h.starts.data(), h.starts.size() * sizeof(int),
                        hipMemcpyHostToDevice));
  return GSWMTP_OK;
}

size_t grouped_bytes(size_t n, size_t item = cgemm_args_bytes()) {
  return align256(item * n) + align256((n + 1) * sizeof(int));
}

// Split-precision products: one plan's whole-tile schedule per item.
GroupedHost build_grouped_split(const std::vector<gswmtp_plan *> &plans,
                                const std::vector<int> &order, bool forward, const GemmTile &tl) {
  const size_t sz = split_args_bytes();
  GroupedHost g;
  g.items.resize(sz * order.size());
  g.starts.resize(order.size() + 1);
  for (size_t k = 0; k < order.size(); ++k) {
    g.starts[k] = g.blocks;
    g.blocks += fill_split_args(plans[order[k]], forward, tl, true, g.items.data() + k * sz);
  }
  g.starts[order.size()] = g.blocks;
  return g;
}

// Split-precision tiles: the product loops of the single-plan form (the
// software-pipelined loop for two terms, two k-groups for three), 64 x 64,
// or a 64 x 128 forward tile (two terms) when GSWMTP_BATCH_TILE=64x128 asks
// and it divides every plan.
int choose_split_tile(gswmtp_batch *b, bool forward, GemmTile &t) {
  const int nt = split_terms_of(b->precision);
  t = GemmTile{64, 64, 32, nt > 2 ? 2 : 1, nt > 2 ? 0 : 1};
  if (nt > 2) {
    if (tile_valid(b->plans, forward, 64, 64)) return GSWMTP_OK;
    return bfail(b, GSWMTP_E_INVAL, "no split tile divides every plan");
  }
  const bool v64 = tile_valid(b->plans, forward, 64, 64);
  const bool v128 = tile_valid(b->plans, forward, 64, 128);
  const char *env = std::getenv("GSWMTP_BATCH_TILE");
  if (env && std::strcmp(env, "64x128") == 0 && v128) {
    t.bn = 128;
    return GSWMTP_OK;
  }
  if (v64) return GSWMTP_OK;
  if (v128) {
    t.bn = 128;
    return GSWMTP_OK;
  }
  return bfail(b, GSWMTP_E_INVAL, "no split tile divides every plan");
}

// Autotuning: among the tiles valid for every plan, the one with the lowest
// mean duration of the grouped product (a few timed launches each).  Only
// run when more than one tile is valid; GSWMTP_BATCH_TILE=BMxBN fixes it.
int choose_batch_tile(gswmtp_batch *b, bool forward, const std::vector<int> &order, int &bm,
                      int &bn) {
  const int dir = forward ? 0 : 1;
  std::vector<int> valid;
  for (int c = 0; c < 4; ++c)
    if (tile_valid(b->plans, forward, kCand[c][0], kCand[c][1])) valid.push_back(c);
  if (valid.empty()) return bfail(b, GSWMTP_E_INVAL, "no tile divides every plan");
  const char *env = std::getenv("GSWMTP_BATCH_TILE");
  if (env) {
    int ebm = 0, ebn = 0;
    if (std::sscanf(env, "%dx%d", &ebm, &ebn) == 2)
      for (int c : valid)
        if (kCand[c][0] == ebm && kCand[c][1] == ebn) {
          bm = ebm;
          bn = ebn;
          return GSWMTP_OK;
        }
  }
  bm = kCand[valid[0]][0];
  bn = kCand[valid[0]][1];
  const char *nt = std::getenv("GSWMTP_BATCH_NO_TUNE");
  if (valid.size() == 1 || (nt && std::atoi(nt) != 0)) return GSWMTP_OK;

  const size_t need = grouped_bytes(b->plans.size());
  size_t sbytes = 0;
  if (!forward)
    for (const auto *p : b->plans) sbytes += 2 * (size_t)p->d.Rp * p->d.Cp * sizeof(float);
  void *tmp = nullptr;
  BHIP_TRY(b, hipMalloc(&tmp, need + sbytes));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = GSWMTP_OK;
  float best = 0.f;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  for (size_t vi = 0; vi < valid.size() && he == hipSuccess; ++vi) {
    const int c = valid[vi];
    const GroupedHost h = build_grouped(b->plans, order, forward, kCand[c][0], kCand[c][1], true,
                                        reinterpret_cast<float *>(static_cast<char *>(tmp) + need));
    char *base = static_cast<char *>(tmp);
    GroupedLaunch g;
    g.bm = kCand[c][0];
    g.bn = kCand[c][1];
    g.epi = forward ? EPI_GATHER : EPI_PROJECT;
    if ((rc = upload_grouped(b, h, base, g)) != GSWMTP_OK) break;
    constexpr int kReps = 4;
    if ((he = launch_cgemm_grouped(g, b->stream)) != hipSuccess) break;   // warm-up
    if ((he = hipEventRecord(e0, b->stream)) != hipSuccess) break;
    for (int r = 0; r < kReps && he == hipSuccess; ++r) he = launch_cgemm_grouped(g, b->stream);
    if (he != hipSuccess) break;
    if ((he = hipEventRecord(e1, b->stream)) != hipSuccess) break;
    if ((he = hipEventSynchronize(e1)) != hipSuccess) break;
    float ms = 0.f;
    if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
    ms /= kReps;
    b->tune_ms[dir][c] = ms;
    if (vi == 0 || ms < best) {
      best = ms;
      bm = g.bm;
      bn = g.bn;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(b->stream);
  (void)hipFree(tmp);
  if (rc != GSWMTP_OK) return rc;
  if (he != hipSuccess) return bfail(b, GSWMTP_E_HIP, "batch tile tuning", he);
  return GSWMTP_OK;
}

int batch_build(gswmtp_batch *b) {
  const int n = (int)b->plans.size();
  BHIP_TRY(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
  BHIP_TRY(b, hipEventCreateWithFlags(&b->ev_user, hipEventDisableTiming));
  BHIP_TRY(b, hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming));
  b->ev_plan.assign(n, nullptr);
  for (auto &e : b->ev_plan) BHIP_TRY(b, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  // plan-time work of every plan precedes anything the batch launches
  for (auto *p : b->plans) BHIP_TRY(b, hipStreamSynchronize(p->stream));

  // dispatch order: longest tiles (largest K) first
  std::vector<int> ofwd(n), obwd(n);
  std::iota(ofwd.begin(), ofwd.end(), 0);
  std::iota(obwd.begin(), obwd.end(), 0);
  std::stable_sort(ofwd.begin(), ofwd.end(),
                   [&](int x, int y) { return b->plans[x]->d.Rp > b->plans[y]->d.Rp; });
  std::stable_sort(obwd.begin(), obwd.end(),
                   [&](int x, int y) { return b->plans[x]->d.Urp > b->plans[y]->d.Urp; });

  int rc;
  const bool split = b->precision != GSWMTP_FP32;
  if (split) {
    if ((rc = choose_split_tile(b, true, b->fwd.tile)) != GSWMTP_OK) return rc;
    if ((rc = choose_split_tile(b, false, b->bwd.tile)) != GSWMTP_OK) return rc;
    b->fwd.bm = b->fwd.tile.bm;
    b->fwd.bn = b->fwd.tile.bn;
    b->bwd.bm = b->bwd.tile.bm;
    b->bwd.bn = b->bwd.tile.bn;
    b->fwd.precision = b->bwd.precision = b->precision;
  } else {
    if ((rc = choose_batch_tile(b, true, ofwd, b->fwd.bm, b->fwd.bn)) != GSWMTP_OK) return rc;
    if ((rc = choose_batch_tile(b, false, obwd, b->bwd.bm, b->bwd.bn)) != GSWMTP_OK) return rc;
  }
  b->fwd.epi = EPI_GATHER;
  b->bwd.epi = EPI_PROJECT;

  // update / scatter items in plan order; the many-focus plans' update
  // items also go to a second table for the update's phases 2 and 3
  const size_t usz = update_args_bytes();
  const size_t ssz = split ? scatter_split_args_bytes() : scatter_args_bytes();
  std::vector<unsigned char> upd(usz * n), sc(ssz * n), big;
  std::vector<int> upd_starts(n + 1), big_starts(1, 0), sc_starts(n + 1);
  std::vector<int *> ctrl(n);
  std::vector<double *> stats(n);
  int blocks = 0, ublocks = 0;
  for (int i = 0; i < n; ++i) {
    gswmtp_plan *p = b->plans[i];
    const int nwg = fill_update_args(p, UPD_ITERATE, b->fwd.bn, upd.data() + i * usz);
    upd_starts[i] = ublocks;
    ublocks += nwg > 0 ? nwg : 1;
    if (nwg > 0) {
      big.insert(big.end(), upd.begin() + i * usz, upd.begin() + (i + 1) * usz);
      big_starts.push_back(big_starts.back() + nwg);
    }
    sc_starts[i] = blocks;
    blocks += split ? fill_scatter_split_args(p, sc.data() + i * ssz)
                    : fill_scatter_args(p, sc.data() + i * ssz);
    ctrl[i] = p->b.ctrl;
    stats[i] = p->b.stats;
  }
  upd_starts[n] = ublocks;
  sc_starts[n] = blocks;
  b->sc_blocks = blocks;
  const int nb = (int)big_starts.size() - 1;

  const size_t isz = split ? split_args_bytes() : cgemm_args_bytes();
  const size_t bytes = 2 * grouped_bytes(n, isz) + align256(usz * n) + align256(ssz * n) +
                       2 * align256((n + 1) * sizeof(int)) + 2 * align256(n * sizeof(void *)) +
                       align256(usz * (nb > 0 ? nb : 1)) + align256((nb + 1) * sizeof(int));
  BHIP_TRY(b, hipMalloc(&b->pool, bytes));
  char *base = static_cast<char *>(b->pool);
  const GroupedHost hf =
      split ? build_grouped_split(b->plans, ofwd, true, b->fwd.tile)
            : build_grouped(b->plans, ofwd, true, b->fwd.bm, b->fwd.bn, false, nullptr);
  const GroupedHost hb =
      split ? build_grouped_split(b->plans, obwd, false, b->bwd.tile)
            : build_grouped(b->plans, obwd, false, b->bwd.bm, b->bwd.bn, false, nullptr);
  if ((rc = upload_grouped(b, hf, base, b->fwd)) != GSWMTP_OK) return rc;
  if ((rc = upload_grouped(b, hb, base, b->bwd)) != GSWMTP_OK) return rc;
  b->upd.d_items = base;
  base += align256(usz * n);
  b->upd.d_starts = reinterpret_cast<int *>(base);
  base += align256((n + 1) * sizeof(int));
  b->upd.n_items = n;
  b->upd.blocks = ublocks;
  b->upd.d_big = base;
  base += align256(usz * (nb > 0 ? nb : 1));
  b->upd.d_big_starts = reinterpret_cast<int *>(base);
  base += align256((nb + 1) * sizeof(int));
  b->upd.n_big = nb;
  b->upd.big_blocks = big_starts.back();
  b->d_sc = base;
  base += align256(ssz * n);
  b->d_sc_starts = reinterpret_cast<int *>(base);
  base += align256((n + 1) * sizeof(int));
  b->d_ctrl = reinterpret_cast<int **>(base);
  base += align256(n * sizeof(void *));
  b->d_stats = reinterpret_cast<double **>(base);
  BHIP_TRY(b, hipMemcpy(b->upd.d_items, upd.data(), upd.size(), hipMemcpyHostToDevice));
  BHIP_TRY(b, hipMemcpy(b->upd.d_starts, upd_starts.data(), upd_starts.size() * sizeof(int),
                        hipMemcpyHostToDevice));
  if (nb > 0) {
    BHIP_TRY(b, hipMemcpy(b->upd.d_big, big.data(), big.size(), hipMemcpyHostToDevice));
    BHIP_TRY(b, hipMemcpy(b->upd.d_big_starts, big_starts.data(), big_starts.size() * sizeof(int),
                          hipMemcpyHostToDevice));
  }
  BHIP_TRY(b, hipMemcpy(b->d_sc, sc.data(), sc.size(), hipMemcpyHostToDevice));
  BHIP_TRY(b, hipMemcpy(b->d_sc_starts, sc_starts.data(), sc_starts.size() * sizeof(int),
                        hipMemcpyHostToDevice));
  BHIP_TRY(b, hipMemcpy(b->d_ctrl, ctrl.data(), n * sizeof(void *), hipMemcpyHostToDevice));
  BHIP_TRY(b, hipMemcpy(b->d_stats, stats.data(), n * sizeof(void *), hipMemcpyHostToDevice));
  return GSWMTP_OK;
}

}  // namespace

extern "C" {

const char *gswmtp_batch_last_error(const gswmtp_batch *b) {
  return b ? b->err.c_str() : g_batch_create_error.c_str();
}

int gswmtp_batch_create(gswmtp_batch **out, gswmtp_plan *const *plans, int n_plans,
                        void *stream) {
  if (!out) return GSWMTP_E_INVAL;
  *out = nullptr;
  g_batch_create_error.clear();
  if (!plans || n_plans < 1 || n_plans > 65536) {
    g_batch_create_error = "batch needs 1..65536 plans";
    return GSWMTP_E_INVAL;
  }
  std::vector<gswmtp_plan *> ps(plans, plans + n_plans);
  for (auto *p : ps) {
    if (!p) {
      g_batch_create_error = "NULL plan";
      return GSWMTP_E_INVAL;
    }
    if (p->precision != ps[0]->precision) {
      g_batch_create_error = "batched plans must share one precision";
      return GSWMTP_E_INVAL;
    }
    if (p->device != ps[0]->device) {
      g_batch_create_error = "batched plans must share one device";
      return GSWMTP_E_INVAL;
    }
  }
  {
    std::vector<gswmtp_plan *> s = ps;
    std::sort(s.begin(), s.end());
    if (std::adjacent_find(s.begin(), s.end()) != s.end()) {
      g_batch_create_error = "a plan appears twice in the batch";
      return GSWMTP_E_INVAL;
    }
  }
  gswmtp_batch *b = new (std::nothrow) gswmtp_batch();
  if (!b) return GSWMTP_E_NOMEM;
  b->device = ps[0]->device;
  b->precision = ps[0]->precision;
  b->user_stream = static_cast<hipStream_t>(stream);
  b->plans = ps;
  const char *ng = std::getenv("GSWMTP_NO_GRAPH");
  b->use_graph = !(ng && std::atoi(ng) != 0);
  DeviceGuardB guard(b->device);
  int rc = batch_build(b);
  if (rc != GSWMTP_OK) {
    g_batch_create_error = b->err;
    free_batch(b);
    return rc;
  }
  *out = b;
  return GSWMTP_OK;
}

int gswmtp_batch_iterate(gswmtp_batch *b, int n_iter, double stop_accuracy) {
  if (!b || n_iter < 0 || !std::isfinite(stop_accuracy)) return GSWMTP_E_INVAL;
  if (n_iter == 0) return GSWMTP_OK;
  DeviceGuardB guard(b->device);
  const int n = (int)b->plans.size();
  // after the caller's stream and every plan's own queued work
  BHIP_TRY(b, hipEventRecord(b->ev_user, b->user_stream));
  BHIP_TRY(b, hipStreamWaitEvent(b->stream, b->ev_user, 0));
  for (int i = 0; i < n; ++i) {
    BHIP_TRY(b, hipEventRecord(b->ev_plan[i], b->plans[i]->stream));
    BHIP_TRY(b, hipStreamWaitEvent(b->stream, b->ev_plan[i], 0));
  }
  hipLaunchKernelGGL(k_batch_control, dim3((n + 255) / 256), dim3(256), 0, b->stream, b->d_ctrl,
                     b->d_stats, n, stop_accuracy);
  BHIP_TRY(b, hipGetLastError());
  if (b->use_graph) {
    if (!b->graph1) BHIP_TRY(b, capture_batch(b, 1, &b->graph1));
    if (n_iter >= 8 && !b->graph8) BHIP_TRY(b, capture_batch(b, 8, &b->graph8));
    int left = n_iter;
    for (; left >= 8; left -= 8) BHIP_TRY(b, hipGraphLaunch(b->graph8, b->stream));
    for (; left > 0; --left) BHIP_TRY(b, hipGraphLaunch(b->graph1, b->stream));
  } else {
    for (int i = 0; i < n_iter; ++i) BHIP_TRY(b, enqueue_batch_pass(b, b->stream));
  }
  // plan calls and the caller's stream come after the batch's passes
  BHIP_TRY(b, hipEventRecord(b->ev_done, b->stream));
  for (auto *p : b->plans) {
    BHIP_TRY(b, hipStreamWaitEvent(p->stream, b->ev_done, 0));
    p->fwd_valid = false;
  }
  BHIP_TRY(b, hipStreamWaitEvent(b->user_stream, b->ev_done, 0));
  return GSWMTP_OK;
}

int gswmtp_batch_set_stream(gswmtp_batch *b, void *stream) {
  if (!b) return GSWMTP_E_INVAL;
  b->user_stream = static_cast<hipStream_t>(stream);
  return GSWMTP_OK;
}

int gswmtp_batch_sync(gswmtp_batch *b) {
  if (!b) return GSWMTP_E_INVAL;
  DeviceGuardB guard(b->device);
  BHIP_TRY(b, hipStreamSynchronize(b->stream));
  return GSWMTP_OK;
}

int gswmtp_batch_tiles(const gswmtp_batch *b, int *tiles, double *tune_ms) {
  if (!b || !tiles) return GSWMTP_E_INVAL;
  tiles[0] = b->fwd.bm;
  tiles[1] = b->fwd.bn;
  tiles[2] = b->bwd.bm;
  tiles[3] = b->bwd.bn;
  if (tune_ms)
    for (int d = 0; d < 2; ++d)
      for (int c = 0; c < 4; ++c) tune_ms[4 * d + c] = b->tune_ms[d][c];
  return GSWMTP_OK;
}

int gswmtp_batch_destroy(gswmtp_batch *b) {
  if (!b) return GSWMTP_OK;
  DeviceGuardB guard(b->device);
  free_batch(b);
  return GSWMTP_OK;
}

}  // extern "C"
