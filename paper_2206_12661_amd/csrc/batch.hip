// Batched form: several independent plans iterated together.
//
// Products.  Every plan's forward and adjoint product belongs to a shape
// class: (product, padded M, N, K).  Each class has its own kernel
// configuration (tile, loop, K chunks of the forward), chosen by the
// autotuner below; the tiles of every plan of a product, as work units
// (plan, tile, K range), go to a device work list per configuration.  Each
// work list is ONE launch.  A stage with one configuration runs it
// persistently: the units, longest first, are dealt to the resident
// workgroups on the host (each to the least-loaded workgroup so far), and
// every workgroup runs its range of units.  A stage's several configurations
// run as parallel branches of the captured graph with one workgroup per unit
// (longest first), which the hardware dispatcher balances across them.

// Autotuner.  For a class whose configuration is not yet known, every
// candidate valid for its shape is timed on the class's own units, repeated
// until the list fills the chip twice (so each candidate is judged on its
// throughput, not on one short launch), with the adjoint's output sent to
// scratch and the done flags ignored, so no plan state changes; the fastest
// wins.  Choices are kept per process and, when GSWMTP_TUNE_CACHE names a
// file, in that JSON file, keyed by architecture, CU count, precision,
// product and (M, N, K).  GSWMTP_BATCH_TILE=BMxBN fixes the tile of every
// class it divides (no tuning); GSWMTP_BATCH_TILE=plan, or
// GSWMTP_BATCH_NO_TUNE=1, gives each class its plans' single-plan
// configuration (no K split).  GSWMTP_BATCH_PERSIST=0 launches one
// workgroup per unit instead of the persistent grid.
//
// The other stages (focus update, scatter) are one grouped launch each over
// all plans.  A pass of the batch is replayed from a captured HIP graph.
//
// Each plan's own arithmetic is exactly that of its single-plan pass with the
// same tile and loop and no K split: a batched result then equals the
// single-plan result bit for bit.  Forward K chunks add their focus-gather
// partials in the focus update like column tiles (fixed order).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <numeric>
#include <queue>
#include <string>
#include <tuple>
#include <vector>

#include "gswmtp_internal.h"

using namespace gswmtp;

// One shape class of a product and its configuration.
struct BatchClass {
  int product = 0;                  // 0 forward (with the focus gather), 1 adjoint
  int M = 0, N = 0, K = 0;          // padded product sizes
  std::vector<int> plans;           // indices into the batch's plans
  WorkConfig cfg;
  double ms = 0.0;                  // timed ms of one copy of its units (0: not timed)
  int source = 0;                   // gswmtp_batch_class::source
  std::vector<std::pair<WorkConfig, double>> tried;   // the tuning table
};

constexpr int kBatchBranches = 4;   // parallel branches per stage beyond the main stream

struct gswmtp_batch {
  int device = 0;
  int cus = 256;
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t side[kBatchBranches] = {};
  hipEvent_t ev_user = nullptr, ev_done = nullptr, ev_fork = nullptr;
  hipEvent_t ev_join[kBatchBranches] = {};
  std::vector<gswmtp_plan *> plans;
  std::vector<hipEvent_t> ev_plan;
  std::vector<BatchClass> classes;
  std::vector<WorkLaunch> work[2];  // per product: one launch per configuration
  GroupedUpdate upd;
  void *d_sc = nullptr;
  int *d_sc_starts = nullptr;
  int sc_blocks = 0;
  int **d_ctrl = nullptr;
  double **d_stats = nullptr;
  void *pool = nullptr;
  hipGraphExec_t graph1 = nullptr, graph8 = nullptr;
  bool use_graph = true;
  bool persistent = true;
  double tune_total_ms = 0.0;       // host time spent timing candidates
  int precision = GSWMTP_FP32;      // common precision of the plans
  int fault_alloc = -1;             // allocation fault injection (fault_alloc_setting)
  int n_alloc = 0;                  // device allocations made by the create call
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

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

bool is_split_prec(int precision) { return split_terms_of(precision) > 0; }

// ---------------------------------------------------------------------------
// Configurations
// ---------------------------------------------------------------------------

// K stages of a configuration's tile for a product of depth K.
int stages_of(const WorkConfig &c, int K) { return K / c.tile.bk; }

// Candidates valid for a class: float32 tiles 64/128 x 64/128 (K stages of
// 16); two-term split tiles 64 x 64 and 64 x 128 on the software-pipelined
// loop and the 16x16-block loop (forward 64 x 128, adjoint 48 x 192);
// three-term split 64 x 64 with two k-groups.  The forward also tries two K
// chunks per 128-wide tile (their gather partials fit the plan's partial
// rows: at most one per 64 columns).
std::vector<WorkConfig> candidates(int precision, int product, int M, int N) {
  std::vector<WorkConfig> out;
  const int nt = split_terms_of(precision);
  auto add = [&](GemmTile t, int split) {
    if (M % t.bm || N % t.bn) return;
    if (split > 1 && (product != 0 || t.bn / 64 < split || t.pipe == 3)) return;
    WorkConfig c;
    c.tile = t;
    c.split = split;
    out.push_back(c);
  };
  if (nt == 0) {
    const int tiles[4][2] = {{64, 64}, {64, 128}, {128, 64}, {128, 128}};
    for (auto &t : tiles) {
      add(GemmTile{t[0], t[1], 16, 1, 0}, 1);
      add(GemmTile{t[0], t[1], 16, 1, 0}, 2);
    }
  } else if (nt == 2) {
    add(GemmTile{64, 64, 32, 1, 1}, 1);
    add(GemmTile{64, 128, 32, 1, 1}, 1);
    add(GemmTile{64, 128, 32, 1, 1}, 2);
    if (product == 0) add(GemmTile{64, 128, 32, 1, 3}, 1);
    else add(GemmTile{48, 192, 32, 1, 3}, 1);
    add(GemmTile{64, 64, 32, 1, 3}, 1);    // 16x16-block loop on the small tiles
  } else {
    add(GemmTile{64, 64, 32, 2, 0}, 1);
  }
  return out;
}

// The plan's own single-plan configuration of a product, without K split.
WorkConfig plan_config(const gswmtp_plan *p, int product) {
  WorkConfig c;
  c.tile = product == 0 ? p->sched_fwd.tile : p->sched_bwd.tile;
  c.split = 1;
  return c;
}

// GSWMTP_BATCH_TILE=BMxBN as a configuration for this precision and product.
bool env_tile(int precision, int product, int M, int N, WorkConfig &c) {
  const char *env = std::getenv("GSWMTP_BATCH_TILE");
  int bm = 0, bn = 0;
  if (!env || std::sscanf(env, "%dx%d", &bm, &bn) != 2) return false;
  const int nt = split_terms_of(precision);
  if (M % bm || N % bn) return false;
  if (nt == 0) {
    if ((bm != 64 && bm != 128) || (bn != 64 && bn != 128)) return false;
    c.tile = GemmTile{bm, bn, 16, 1, 0};
  } else if (nt == 2) {
    if (bm != 64 || (bn != 64 && bn != 128)) return false;
    c.tile = GemmTile{64, bn, 32, 1, 1};
  } else {
    if (bm != 64 || bn != 64) return false;
    c.tile = GemmTile{64, 64, 32, 2, 0};
  }
  c.split = 1;
  (void)product;
  return true;
}

std::string config_text(const WorkConfig &c) {
  char buf[64];
  snprintf(buf, sizeof buf, "%dx%d/%s/k%d", c.tile.bm, c.tile.bn,
           c.tile.pipe == 3 ? "b16" : c.tile.kg == 2 ? "kg2" : c.tile.pipe == 2 ? "direct"
                              : c.tile.pipe == 1 ? "pipe" : "plain",
           c.split);
  return buf;
}

// ---------------------------------------------------------------------------
// Tuning cache: per process, and in the JSON file GSWMTP_TUNE_CACHE names.
// The file is one object of entries, one per line,
//   "arch:cus:precision:product:MxNxK": [[bm, bn, bk, kgroups, loop, split, ms], ...]
// holding the timed candidates of the class (its tuning table).
// ---------------------------------------------------------------------------

typedef std::vector<std::pair<WorkConfig, double>> TuneTable;
std::mutex g_cache_mu;
std::map<std::string, TuneTable> g_cache;

const char *prec_name(int precision) {
  switch (precision) {
    case GSWMTP_BF16X3: return "bf16x3";
    case GSWMTP_FP16X3: return "fp16x3";
    case GSWMTP_BF16X6: return "bf16x6";
  }
  return "fp32";
}

std::string cache_key(const std::string &arch, int cus, int precision, const BatchClass &c) {
  char buf[160];
  snprintf(buf, sizeof buf, "%s:%d:%s:%s:%dx%dx%d", arch.c_str(), cus, prec_name(precision),
           c.product == 0 ? "forward" : "adjoint", c.M, c.N, c.K);
  return buf;
}

void cache_load(const char *path) {
  std::ifstream in(path);
  if (!in) return;
  std::string line;
  while (std::getline(in, line)) {
    const size_t q0 = line.find('"'), q1 = line.find('"', q0 + 1);
    if (q0 == std::string::npos || q1 == std::string::npos) continue;
    TuneTable t;
    size_t at = line.find('[', q1);
    if (at == std::string::npos) continue;
    for (at = line.find('[', at + 1); at != std::string::npos; at = line.find('[', at + 1)) {
      WorkConfig c;
      double ms = 0.0;
      if (std::sscanf(line.c_str() + at, "[%d, %d, %d, %d, %d, %d, %lf]", &c.tile.bm, &c.tile.bn,
                      &c.tile.bk, &c.tile.kg, &c.tile.pipe, &c.split, &ms) != 7)
        break;
      t.push_back({c, ms});
    }
    if (!t.empty()) g_cache[line.substr(q0 + 1, q1 - q0 - 1)] = t;
  }
}

bool cache_save(const char *path) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp);
    if (!out) return false;
    out << "{\n";
    size_t k = 0;
    for (const auto &e : g_cache) {
      out << "  \"" << e.first << "\": [";
      for (size_t i = 0; i < e.second.size(); ++i) {
        const WorkConfig &c = e.second[i].first;
        // times with every digit a double holds: the choice made from the
        // table read back (the fastest, then the 10% rule below) must be the
        // tuning run's, also for near-equal candidates
        char buf[128];
        snprintf(buf, sizeof buf, "[%d, %d, %d, %d, %d, %d, %.17g]", c.tile.bm, c.tile.bn,
                 c.tile.bk, c.tile.kg, c.tile.pipe, c.split, e.second[i].second);
        out << (i ? ", " : "") << buf;
      }
      out << "]" << (++k < g_cache.size() ? ",\n" : "\n");
    }
    out << "}\n";
    if (!out) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

// The fastest entry of a tuning table (the first of equal times).
void take_best(BatchClass &cl) {
  for (size_t i = 0; i < cl.tried.size(); ++i)
    if (i == 0 || cl.tried[i].second < cl.ms) {
      cl.cfg = cl.tried[i].first;
      cl.ms = cl.tried[i].second;
    }
}

// ---------------------------------------------------------------------------
// Work lists
// ---------------------------------------------------------------------------

// Units of one plan's product under configuration c (item k of the launch).
void add_units(std::vector<WorkUnit> &u, int item, int tiles, int tiles_m, int K,
               const WorkConfig &c) {
  const int KT = stages_of(c, K), tiles_n = tiles / tiles_m;
  for (int t = 0; t < tiles; ++t)
    for (int ch = 0; ch < c.split; ++ch) {
      WorkUnit w{};
      w.item = item;
      w.tile = t;
      w.kb = ch * KT / c.split;
      w.ke = (ch + 1) * KT / c.split;
      w.prow = ch * tiles_n + t / tiles_m;
      u.push_back(w);
    }
}

// Longest units first (K stages, then plan and tile order).
void sort_units(std::vector<WorkUnit> &u) {
  std::stable_sort(u.begin(), u.end(),
                   [](const WorkUnit &x, const WorkUnit &y) { return x.ke - x.kb > y.ke - y.kb; });
}

// Estimated cost of a unit in K stages, with a fixed per-unit share for its
// prologue and epilogue.
double unit_cost(const WorkUnit &u) { return (double)(u.ke - u.kb) + 4.0; }

// Persistent grid: the units (longest first) dealt to `grid` workgroups, each
// to the least-loaded one so far (longest-processing-time list scheduling);
// u is reordered by workgroup and off[b] .. off[b + 1] - 1 are workgroup b's.
void assign_units(std::vector<WorkUnit> &u, int grid, std::vector<int> &off) {
  typedef std::pair<double, int> Load;   // (cost so far, workgroup)
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (int b = 0; b < grid; ++b) heap.push({0.0, b});
  std::vector<std::vector<WorkUnit>> per(grid);
  for (const auto &w : u) {
    Load l = heap.top();
    heap.pop();
    per[l.second].push_back(w);
    l.first += unit_cost(w);
    heap.push(l);
  }
  off.assign(grid + 1, 0);
  u.clear();
  for (int b = 0; b < grid; ++b) {
    off[b] = (int)u.size();
    u.insert(u.end(), per[b].begin(), per[b].end());
  }
  off[grid] = (int)u.size();
}


int occupancy(const gswmtp_batch *b, const WorkConfig &c, int epi) {
  const int n = is_split_prec(b->precision) ? cgemm_split_work_occupancy(c, epi, b->precision)
                                             : cgemm_work_occupancy(c, epi);
  return n > 0 ? n : 1;
}

hipError_t launch_work(const gswmtp_batch *b, const WorkLaunch &w, hipStream_t s) {
  return is_split_prec(b->precision) ? launch_cgemm_split_work(w, s) : launch_cgemm_work(w, s);
}

// Product arguments of plan p under configuration c.  out_cr / out_ci /
// out_pt (tuning): the adjoint's output redirected.
int fill_item(const gswmtp_batch *b, const gswmtp_plan *p, int product, const WorkConfig &c,
              bool honour_done, float *out_cr, float *out_ci, unsigned short *out_pt,
              void *out) {
  if (is_split_prec(b->precision))
    return fill_split_args(p, product == 0, c.tile, honour_done, out_pt, out);
  return fill_cgemm_args(p, product == 0, c.tile.bm, c.tile.bn, honour_done, out_cr, out_ci,
                         out);
}

size_t item_bytes(const gswmtp_batch *b) {
  return is_split_prec(b->precision) ? split_args_bytes() : cgemm_args_bytes();
}

// ---------------------------------------------------------------------------
// Autotuning of one class
// ---------------------------------------------------------------------------

struct TuneScratch {
  void *buf = nullptr;
  size_t bytes = 0;
  ~TuneScratch() {
    if (buf) (void)hipFree(buf);
  }
  hipError_t need(size_t n) {
    if (n <= bytes) return hipSuccess;
    if (buf) (void)hipFree(buf);
    buf = nullptr;
    bytes = 0;
    const hipError_t e = hipMalloc(&buf, n);
    if (e == hipSuccess) bytes = n;
    return e;
  }
};

int tune_class(gswmtp_batch *b, BatchClass &cl, TuneScratch &ts) {
  const std::vector<WorkConfig> cands = candidates(b->precision, cl.product, cl.M, cl.N);
  const int epi = cl.product == 0 ? EPI_GATHER : EPI_PROJECT;
  const size_t isz = item_bytes(b);
  const int np = (int)cl.plans.size();
  const bool split = is_split_prec(b->precision);
  // adjoint output redirected to scratch: per plan [Rp][Cp] float planes, or
  // the split planes of P^T
  std::vector<size_t> out_off(np, 0);
  size_t out_bytes = 0;
  for (int k = 0; k < np; ++k) {
    const gswmtp_plan *p = b->plans[cl.plans[k]];
    const size_t plane = (size_t)p->d.Rp * p->d.Cp;
    out_off[k] = out_bytes;
    if (cl.product == 1)
      out_bytes += align256(split ? 2 * (size_t)split_terms_of(b->precision) * plane * 2
                                  : 2 * plane * sizeof(float));
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BHIP_TRY(b, hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return bfail(b, GSWMTP_E_HIP, "tuning events", he);
  }
  int rc = GSWMTP_OK;
  for (size_t ci = 0; ci < cands.size() && rc == GSWMTP_OK; ++ci) {
    const WorkConfig &c = cands[ci];
    // the class's units, repeated until they fill the chip twice
    std::vector<WorkUnit> units;
    for (int k = 0; k < np; ++k) {
      const gswmtp_plan *p = b->plans[cl.plans[k]];
      const int tiles_m = (cl.product == 0 ? p->d.Urp : p->d.Rp) / c.tile.bm;
      add_units(units, k, tiles_m * (p->d.Cp / c.tile.bn), tiles_m, cl.K, c);
    }
    const int slots = b->cus * occupancy(b, c, epi);
    const int one = (int)units.size();
    const int reps = std::max(1, (2 * slots + one - 1) / one);
    std::vector<WorkUnit> all;
    all.reserve((size_t)one * reps);
    for (int r = 0; r < reps; ++r) all.insert(all.end(), units.begin(), units.end());
    const int grid = b->persistent ? std::min((int)all.size(), slots) : (int)all.size();
    std::vector<int> off;
    if (b->persistent) assign_units(all, grid, off);
    // scratch: [adjoint outputs][items][units][unit ranges]
    const size_t need = align256(out_bytes) + align256(isz * np) +
                        align256(all.size() * sizeof(WorkUnit)) +
                        align256(off.size() * sizeof(int));
    if (need > ts.bytes && fault_alloc_hit(b->fault_alloc, &b->n_alloc)) {
      rc = bfail(b, GSWMTP_E_NOMEM, "batch tuning scratch: injected failure");
      break;
    }
    if ((he = ts.need(need)) != hipSuccess) {
      rc = bfail(b, GSWMTP_E_NOMEM, "batch tuning scratch", he);
      break;
    }
    char *base = static_cast<char *>(ts.buf);
    std::vector<unsigned char> items(isz * np);
    for (int k = 0; k < np; ++k) {
      const gswmtp_plan *p = b->plans[cl.plans[k]];
      const size_t plane = (size_t)p->d.Rp * p->d.Cp;
      char *o = base + out_off[k];
      float *cr = nullptr, *cim = nullptr;
      unsigned short *pt = nullptr;
      if (cl.product == 1) {
        if (split) {
          pt = reinterpret_cast<unsigned short *>(o);
        } else {
          cr = reinterpret_cast<float *>(o);
          cim = cr + plane;
        }
      }
      fill_item(b, p, cl.product, c, false, cr, cim, pt, items.data() + k * isz);
    }
    char *d_items = base + align256(out_bytes);
    WorkUnit *d_work = reinterpret_cast<WorkUnit *>(d_items + align256(items.size()));
    int *d_off = reinterpret_cast<int *>(reinterpret_cast<char *>(d_work) +
                                         align256(all.size() * sizeof(WorkUnit)));
    if ((he = hipMemcpy(d_items, items.data(), items.size(), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (he = hipMemcpy(d_work, all.data(), all.size() * sizeof(WorkUnit),
                        hipMemcpyHostToDevice)) != hipSuccess ||
        (!off.empty() && (he = hipMemcpy(d_off, off.data(), off.size() * sizeof(int),
                                         hipMemcpyHostToDevice)) != hipSuccess)) {
      rc = bfail(b, GSWMTP_E_HIP, "batch tuning upload", he);
      break;
    }
    WorkLaunch w;
    w.cfg = c;
    w.epi = epi;
    w.precision = b->precision;
    w.d_items = d_items;
    w.d_work = d_work;
    w.d_off = off.empty() ? nullptr : d_off;
    w.n_work = (int)all.size();
    w.grid = grid;
    constexpr int kReps = 3;
    if ((he = launch_work(b, w, b->stream)) != hipSuccess ||   // warm-up
        (he = hipEventRecord(e0, b->stream)) != hipSuccess) {
      rc = bfail(b, GSWMTP_E_HIP, "batch tuning launch", he);
      break;
    }
    for (int r = 0; r < kReps && he == hipSuccess; ++r) he = launch_work(b, w, b->stream);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventRecord(e1, b->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) {
      rc = bfail(b, GSWMTP_E_HIP, "batch tuning launch", he);
      break;
    }
    cl.tried.push_back({c, (double)ms / kReps / reps});   // one copy of the class's units
  }
  (void)hipStreamSynchronize(b->stream);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

// ---------------------------------------------------------------------------
// Stages of a batched pass
// ---------------------------------------------------------------------------

// One product: its configurations' launches, the first on `s`, the others
// as parallel branches forked from `s` and joined back to it.
hipError_t enqueue_product(gswmtp_batch *b, int product, hipStream_t s) {
  const std::vector<WorkLaunch> &ws = b->work[product];
  if (ws.empty()) return hipSuccess;
  hipError_t e;
  const int side = (int)ws.size() - 1;
  if (side > 0) {
    if ((e = hipEventRecord(b->ev_fork, s)) != hipSuccess) return e;
    for (int k = 0; k < side; ++k)
      if ((e = hipStreamWaitEvent(b->side[k], b->ev_fork, 0)) != hipSuccess) return e;
  }
  if ((e = launch_work(b, ws[0], s)) != hipSuccess) return e;
  for (int k = 0; k < side; ++k) {
    if ((e = launch_work(b, ws[k + 1], b->side[k])) != hipSuccess) return e;
    if ((e = hipEventRecord(b->ev_join[k], b->side[k])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, b->ev_join[k], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t enqueue_batch_pass(gswmtp_batch *b, hipStream_t s) {
  hipError_t e;
  const int n = (int)b->plans.size();
  if ((e = enqueue_product(b, 0, s)) != hipSuccess) return e;
  if ((e = launch_update_grouped(b->upd, s)) != hipSuccess) return e;
  if (is_split_prec(b->precision)) {
    if ((e = launch_scatter_split_grouped(b->d_sc, b->d_sc_starts, n, b->sc_blocks, b->precision,
                                          s)) != hipSuccess)
      return e;
  } else {
    if ((e = launch_scatter_grouped(b->d_sc, b->d_sc_starts, n, b->sc_blocks, s)) != hipSuccess)
      return e;
  }
  return enqueue_product(b, 1, s);
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
  for (auto st : b->side)
    if (st) (void)hipStreamSynchronize(st);
  if (b->graph1) (void)hipGraphExecDestroy(b->graph1);
  if (b->graph8) (void)hipGraphExecDestroy(b->graph8);
  if (b->pool) (void)hipFree(b->pool);
  for (auto e : b->ev_plan)
    if (e) (void)hipEventDestroy(e);
  for (auto e : b->ev_join)
    if (e) (void)hipEventDestroy(e);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_user) (void)hipEventDestroy(b->ev_user);
  if (b->ev_done) (void)hipEventDestroy(b->ev_done);
  for (auto st : b->side)
    if (st) (void)hipStreamDestroy(st);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

// Shape classes of both products, in first-appearance order.
void make_classes(gswmtp_batch *b) {
  std::map<std::tuple<int, int, int, int>, int> index;
  for (int i = 0; i < (int)b->plans.size(); ++i) {
    const Dims &d = b->plans[i]->d;
    for (int product = 0; product < 2; ++product) {
      const int M = product == 0 ? d.Urp : d.Rp, N = d.Cp, K = product == 0 ? d.Rp : d.Urp;
      const auto key = std::make_tuple(product, M, N, K);
      auto it = index.find(key);
      if (it == index.end()) {
        BatchClass c;
        c.product = product;
        c.M = M;
        c.N = N;
        c.K = K;
        it = index.emplace(key, (int)b->classes.size()).first;
        b->classes.push_back(c);
      }
      b->classes[it->second].plans.push_back(i);
    }
  }
}

// Configuration of every class: forced, the plans' own, cached or tuned.
int configure_classes(gswmtp_batch *b) {
  const char *tenv = std::getenv("GSWMTP_BATCH_TILE");
  const char *nt = std::getenv("GSWMTP_BATCH_NO_TUNE");
  const bool plan_cfg = (tenv && std::strcmp(tenv, "plan") == 0) || (nt && std::atoi(nt) != 0);
  const char *cpath = std::getenv("GSWMTP_TUNE_CACHE");
  hipDeviceProp_t prop;
  BHIP_TRY(b, hipGetDeviceProperties(&prop, b->device));
  std::string arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  std::lock_guard<std::mutex> lock(g_cache_mu);
  if (cpath && *cpath) cache_load(cpath);
  TuneScratch ts;
  bool tuned = false;
  for (auto &cl : b->classes) {
    const gswmtp_plan *p0 = b->plans[cl.plans[0]];
    WorkConfig forced;
    if (env_tile(b->precision, cl.product, cl.M, cl.N, forced)) {
      cl.cfg = forced;
      cl.source = 3;
      continue;
    }
    const std::vector<WorkConfig> cands = candidates(b->precision, cl.product, cl.M, cl.N);
    if (plan_cfg || cands.size() <= 1) {
      cl.cfg = cands.size() == 1 && !plan_cfg ? cands[0] : plan_config(p0, cl.product);
      cl.source = 0;
      continue;
    }
    const std::string key = cache_key(arch, b->cus, b->precision, cl);
    auto it = g_cache.find(key);
    bool hit = it != g_cache.end();
    if (hit)   // every cached candidate must still be one of this build's
      for (const auto &t : it->second)
        hit = hit && std::find(cands.begin(), cands.end(), t.first) != cands.end();
    if (hit) {
      cl.tried = it->second;
      take_best(cl);
      cl.source = 2;
      continue;
    }
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = tune_class(b, cl, ts);
    b->tune_total_ms +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rc != GSWMTP_OK) return rc;
    take_best(cl);
    cl.source = 1;
    g_cache[key] = cl.tried;
    tuned = true;
  }
  if (tuned && cpath && *cpath && !cache_save(cpath))
    return bfail(b, GSWMTP_E_INVAL, "cannot write the tuning cache (GSWMTP_TUNE_CACHE)");
  // Every extra configuration of a stage is another concurrent launch, which
  // the stage pays for in balance (one workgroup per unit instead of a
  // persistent grid): a tuned class whose timing of the product's dominant
  // configuration (the one with the most padded work) is within 10% of its
  // own best takes the dominant one.
  for (int product = 0; product < 2; ++product) {
    std::vector<std::pair<WorkConfig, double>> work;
    for (const auto &cl : b->classes) {
      if (cl.product != product) continue;
      const double w = (double)cl.M * cl.N * cl.K * cl.plans.size();
      size_t k = 0;
      while (k < work.size() && !(work[k].first == cl.cfg)) ++k;
      if (k == work.size()) work.push_back({cl.cfg, 0.0});
      work[k].second += w;
    }
    if (work.size() < 2) continue;
    const WorkConfig dom = std::max_element(work.begin(), work.end(), [](const auto &x,
                                                                         const auto &y) {
                             return x.second < y.second;
                           })->first;
    for (auto &cl : b->classes) {
      if (cl.product != product || cl.cfg == dom || cl.tried.empty()) continue;
      for (const auto &t : cl.tried)
        if (t.first == dom && t.second <= 1.10 * cl.ms) {
          cl.cfg = dom;
          cl.ms = t.second;
        }
    }
  }
  // GSWMTP_BATCH_FWD_SPLIT=k: k K chunks on every forward class whose tile
  // takes them (k <= BN / 64, not the 16x16-block loop)
  if (const char *fs = std::getenv("GSWMTP_BATCH_FWD_SPLIT")) {
    const int k = std::atoi(fs);
    for (auto &cl : b->classes)
      if (cl.product == 0 && k >= 1 && cl.cfg.tile.pipe != 3 && k <= cl.cfg.tile.bn / 64 &&
          k <= stages_of(cl.cfg, cl.K))
        cl.cfg.split = k;
  }
  return GSWMTP_OK;
}

int batch_build(gswmtp_batch *b) {
  const int n = (int)b->plans.size();
  BHIP_TRY(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
  for (auto &st : b->side) BHIP_TRY(b, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  BHIP_TRY(b, hipEventCreateWithFlags(&b->ev_user, hipEventDisableTiming));
  BHIP_TRY(b, hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming));
  BHIP_TRY(b, hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
  for (auto &e : b->ev_join) BHIP_TRY(b, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  b->ev_plan.assign(n, nullptr);
  for (auto &e : b->ev_plan) BHIP_TRY(b, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  // plan-time work of every plan precedes anything the batch launches
  for (auto *p : b->plans) BHIP_TRY(b, hipStreamSynchronize(p->stream));
  int cus = 0;
  BHIP_TRY(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
  b->cus = cus > 0 ? cus : 256;
  const char *pe = std::getenv("GSWMTP_BATCH_PERSIST");
  b->persistent = !(pe && std::strcmp(pe, "0") == 0);

  make_classes(b);
  int rc;
  if ((rc = configure_classes(b)) != GSWMTP_OK) return rc;

  // per plan: its class configuration of each product
  std::vector<WorkConfig> pcfg[2];
  pcfg[0].resize(n);
  pcfg[1].resize(n);
  for (const auto &cl : b->classes)
    for (int i : cl.plans) pcfg[cl.product][i] = cl.cfg;

  // product items (one per plan and product) and the work lists per configuration
  const size_t isz = item_bytes(b);
  std::vector<unsigned char> items[2];
  std::vector<WorkConfig> cfgs[2];
  std::vector<std::vector<WorkUnit>> units[2];
  for (int product = 0; product < 2; ++product) {
    items[product].resize(isz * n);
    for (int i = 0; i < n; ++i) {
      const gswmtp_plan *p = b->plans[i];
      const WorkConfig &c = pcfg[product][i];
      const int tiles = fill_item(b, p, product, c, true, nullptr, nullptr, nullptr,
                                  items[product].data() + i * isz);
      size_t k = 0;
      while (k < cfgs[product].size() && !(cfgs[product][k] == c)) ++k;
      if (k == cfgs[product].size()) {
        cfgs[product].push_back(c);
        units[product].emplace_back();
      }
      add_units(units[product][k], i, tiles, (product == 0 ? p->d.Urp : p->d.Rp) / c.tile.bm,
                product == 0 ? p->d.Rp : p->d.Urp, c);
    }
    if ((int)cfgs[product].size() > kBatchBranches + 1)
      return bfail(b, GSWMTP_E_UNSUPPORTED, "more kernel configurations than parallel branches");
    // the configuration with most work first (it runs on the main stream)
    std::vector<size_t> ord(cfgs[product].size());
    std::iota(ord.begin(), ord.end(), 0);
    auto work_of = [&](size_t k) {
      double wsum = 0.0;
      for (const auto &u : units[product][k])
        wsum += (double)(u.ke - u.kb) * cfgs[product][k].tile.bm * cfgs[product][k].tile.bn *
                cfgs[product][k].tile.bk;
      return wsum;
    };
    std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return work_of(x) > work_of(y); });
    std::vector<WorkConfig> c2;
    std::vector<std::vector<WorkUnit>> u2;
    for (size_t k : ord) {
      c2.push_back(cfgs[product][k]);
      u2.push_back(std::move(units[product][k]));
      sort_units(u2.back());
    }
    cfgs[product] = c2;
    units[product] = std::move(u2);
  }

  // focus update and scatter items in plan order; the many-focus plans'
  // update items also go to a second table for the update's phases 2 and 3
  const bool split = is_split_prec(b->precision);
  const size_t usz = update_args_bytes();
  const size_t ssz = split ? scatter_split_args_bytes() : scatter_args_bytes();
  std::vector<unsigned char> upd(usz * n), sc(ssz * n), big;
  std::vector<int> upd_starts(n + 1), big_starts(1, 0), sc_starts(n + 1);
  std::vector<int *> ctrl(n);
  std::vector<double *> stats(n);
  int blocks = 0, ublocks = 0;
  for (int i = 0; i < n; ++i) {
    gswmtp_plan *p = b->plans[i];
    const WorkConfig &cf = pcfg[0][i];
    const int nwg = fill_update_args(p, UPD_ITERATE, (p->d.Cp / cf.tile.bn) * cf.split,
                                     upd.data() + i * usz);
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

  // Grids and the persistent launches' unit ranges.
  std::vector<int> grids[2];
  std::vector<std::vector<int>> offs[2];
  for (int product = 0; product < 2; ++product) {
    const int epi = product == 0 ? EPI_GATHER : EPI_PROJECT;
    for (size_t k = 0; k < cfgs[product].size(); ++k) {
      auto &u = units[product][k];
      const int slots = b->cus * occupancy(b, cfgs[product][k], epi);
      int grid = std::max(1, std::min(slots, (int)u.size()));
      std::vector<int> off;
      // persistent when the stage has this configuration alone; several
      // concurrent configurations run one workgroup per unit, which the
      // hardware balances across them (a static split between kernels that
      // share the CUs leaves one waiting on the other)
      if (b->persistent && cfgs[product].size() == 1 && cfgs[product][k].tile.kg == 1) {
        assign_units(u, grid, off);
      } else {
        grid = (int)u.size();   // one unit per workgroup, longest first
      }
      grids[product].push_back(grid);
      offs[product].push_back(off);
    }
  }

  size_t bytes = 2 * align256(isz * n) + align256(usz * n) + align256(ssz * n) +
                 2 * align256((n + 1) * sizeof(int)) + 2 * align256(n * sizeof(void *)) +
                 align256(usz * (nb > 0 ? nb : 1)) + align256((nb + 1) * sizeof(int));
  for (int product = 0; product < 2; ++product)
    for (size_t k = 0; k < units[product].size(); ++k)
      bytes += align256(units[product][k].size() * sizeof(WorkUnit)) +
               align256(offs[product][k].size() * sizeof(int));
  if (fault_alloc_hit(b->fault_alloc, &b->n_alloc))
    return bfail(b, GSWMTP_E_NOMEM, "batch device pool: injected failure");
  BHIP_TRY(b, hipMalloc(&b->pool, bytes));
  char *base = static_cast<char *>(b->pool);
  for (int product = 0; product < 2; ++product) {
    char *d_items = base;
    base += align256(isz * n);
    BHIP_TRY(b, hipMemcpy(d_items, items[product].data(), items[product].size(),
                          hipMemcpyHostToDevice));
    const int epi = product == 0 ? EPI_GATHER : EPI_PROJECT;
    for (size_t k = 0; k < cfgs[product].size(); ++k) {
      const auto &u = units[product][k];
      WorkLaunch w;
      w.cfg = cfgs[product][k];
      w.epi = epi;
      w.precision = b->precision;
      w.d_items = d_items;
      w.d_work = reinterpret_cast<const WorkUnit *>(base);
      w.n_work = (int)u.size();
      w.grid = grids[product][k];
      BHIP_TRY(b, hipMemcpy(base, u.data(), u.size() * sizeof(WorkUnit), hipMemcpyHostToDevice));
      base += align256(u.size() * sizeof(WorkUnit));
      const auto &off = offs[product][k];
      if (!off.empty()) {
        w.d_off = reinterpret_cast<const int *>(base);
        BHIP_TRY(b, hipMemcpy(base, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
        base += align256(off.size() * sizeof(int));
      }
      b->work[product].push_back(w);
    }
  }
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

// The class with the most padded work of a product.
const BatchClass *largest_class(const gswmtp_batch *b, int product) {
  const BatchClass *best = nullptr;
  double bw = -1.0;
  for (const auto &c : b->classes) {
    if (c.product != product) continue;
    const double w = (double)c.M * c.N * c.K * c.plans.size();
    if (w > bw) {
      bw = w;
      best = &c;
    }
  }
  return best;
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
  const int fault = fault_alloc_setting();
  if (fault == 0) {
    g_batch_create_error = "device allocation: injected failure (GSWMTP_FAULT_INJECT=alloc)";
    return GSWMTP_E_NOMEM;
  }
  gswmtp_batch *b = new (std::nothrow) gswmtp_batch();
  if (!b) return GSWMTP_E_NOMEM;
  b->fault_alloc = fault;
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
    p->fwd_valid = p->stats_valid = false;
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
  for (int product = 0; product < 2; ++product) {
    const BatchClass *c = largest_class(b, product);
    tiles[2 * product] = c ? c->cfg.tile.bm : 0;
    tiles[2 * product + 1] = c ? c->cfg.tile.bn : 0;
  }
  if (tune_ms) {
    static const int cand[4][2] = {{64, 64}, {64, 128}, {128, 64}, {128, 128}};
    for (int product = 0; product < 2; ++product) {
      const BatchClass *c = largest_class(b, product);
      for (int k = 0; k < 4; ++k) {
        tune_ms[4 * product + k] = 0.0;
        if (!c) continue;
        for (const auto &t : c->tried)
          if (t.first.tile.bm == cand[k][0] && t.first.tile.bn == cand[k][1] &&
              t.first.split == 1 && t.first.tile.pipe != 3)
            tune_ms[4 * product + k] = t.second;
      }
    }
  }
  return GSWMTP_OK;
}

int gswmtp_batch_n_classes(const gswmtp_batch *b, int *n) {
  if (!b || !n) return GSWMTP_E_INVAL;
  *n = (int)b->classes.size();
  return GSWMTP_OK;
}

int gswmtp_batch_class_info(const gswmtp_batch *b, int i, gswmtp_batch_class *out) {
  if (!b || !out || i < 0 || i >= (int)b->classes.size()) return GSWMTP_E_INVAL;
  const BatchClass &c = b->classes[i];
  std::memset(out, 0, sizeof *out);
  out->product = c.product;
  out->m = c.M;
  out->n = c.N;
  out->k = c.K;
  out->n_plans = (int)c.plans.size();
  auto put = [](const WorkConfig &w, int *cfg) {
    cfg[0] = w.tile.bm;
    cfg[1] = w.tile.bn;
    cfg[2] = w.tile.bk;
    cfg[3] = w.tile.kg;
    cfg[4] = w.tile.pipe;
    cfg[5] = w.split;
  };
  put(c.cfg, out->config);
  out->ms = c.ms;
  out->source = c.source;
  out->n_tried = (int)std::min<size_t>(c.tried.size(), GSWMTP_BATCH_MAX_CANDIDATES);
  for (int k = 0; k < out->n_tried; ++k) {
    put(c.tried[k].first, out->tried_config[k]);
    out->tried_ms[k] = c.tried[k].second;
  }
  return GSWMTP_OK;
}

int gswmtp_batch_tune_ms(const gswmtp_batch *b, double *ms) {
  if (!b || !ms) return GSWMTP_E_INVAL;
  *ms = b->tune_total_ms;
  return GSWMTP_OK;
}

int gswmtp_batch_destroy(gswmtp_batch *b) {
  if (!b) return GSWMTP_OK;
  DeviceGuardB guard(b->device);
  free_batch(b);
  return GSWMTP_OK;
}

}  // extern "C"
