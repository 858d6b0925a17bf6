// Internal declarations of the gfx950 GSW-MTP library (not part of the C ABI).
//
// Layout of a plan on the device ("internal orientation"):
//   The dense complex product of Eq. 2 runs over one focal axis, the "r" axis
//   (y unless x has fewer unique focus coordinates).  Internal pupil row r is
//   the r-th kept pupil row (axis y) or kept pupil column (axis x); internal
//   column c is the other kept pupil coordinate.  Every matrix is stored as two
//   float32 planes (real, imaginary), row-major, zero-padded to tile multiples:
//     P    [Rp][Cp]   pupil field E = A exp(i phi)        (Rk x Ck used)
//     amp  [Rp][Cp]   amplitude, 0 in the padding
//     OmT  [Rp][Urp]  Omega_r^T: OmT[j][a] = exp(-2 pi i s_r ur_j R_a)
//     OmC  [Urp][Rp]  conj(Omega_r):  OmC[a][j] = conj(OmT[j][a])
//     Wc   [Uc][Cp]   Omega_c^T: Wc[b][i] = exp(-2 pi i s_c uc_i C_b)
//     S    [Urp][Cp]  scatter of the new focal field onto its r rows
//   One pass:  L = OmT^T P with Theta_n = sum_i L[ir_n][i] Wc[ic_n][i] formed
//   in the product's epilogue (L is never stored); focus update;
//   S[a][i] = sum_{n: ir_n = a} Theta'_n conj(Wc[ic_n][i]);
//   P = amp * normalise(OmC^T S).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/gswmtp.h"

namespace gswmtp {

constexpr int kHistCap = 4096;     // history ring entries
constexpr int kPadRows = 64;       // padding granule of M / K dimensions

// K-blocked storage of a split operand plane [rows][K] (K a multiple of
// kKB): K / kKB blocks of [rows][kKB], so kKB consecutive k of consecutive
// rows - one product stage of a row tile - are one contiguous run and every
// stage load covers whole cache lines.
constexpr int kKB = 32;
__host__ __device__ __forceinline__ size_t kblk_index(size_t row, size_t k, size_t rows) {
  return (k / kKB) * rows * kKB + row * kKB + (k % kKB);
}
constexpr int kPadCols = 64;       // padding granule of the N dimension
constexpr int kMaxFoci = 262144;
constexpr int kMaxSide = 16384;
constexpr int kApBlocks = 256;          // workgroups of the aperture statistics

// Control block (device ints): done flag, passes done, history count,
// non-finite flag, phase-fixing pass (0: off), phase-fixing phasors recorded.
enum {
  CTRL_DONE = 0, CTRL_ITERS = 1, CTRL_HIST = 2, CTRL_NONFINITE = 3, CTRL_FIX = 4, CTRL_FIXED = 5,
  CTRL_N = 8
};
// Stats block (device doubles): xi, eta, U, sum I, stop threshold, ...
enum { ST_XI = 0, ST_ETA = 1, ST_U = 2, ST_SUMI = 3, ST_STOP = 4, ST_N = 8 };

struct Dims {
  int ny = 0, nx = 0, nf = 0;
  int ux = 0, uy = 0, ny_kept = 0, nx_kept = 0;
  int axis = 0;
  int Rk = 0, Ck = 0, Ur = 0, Uc = 0;   // internal orientation
  int Rp = 0, Cp = 0, Urp = 0;          // padded
  int Ucp = 0;                          // padded Uc (grid form)
  int n_ap = 0;
  double sum_a2 = 0.0;
};

// Device buffers of one plan.
struct Bufs {
  // inputs and index work (sized by ny, nx, nf)
  double *fx = nullptr, *fy = nullptr, *target = nullptr, *tnorm = nullptr;
  double *tinv = nullptr, *tsqrt = nullptr;   // 1 / tnorm (0 at tnorm 0), sqrt(target)
  double *fz = nullptr;                  // axial positions (zeros: the focal plane)
  double *meas = nullptr;                // [nf] measured intensities, then at unit sum
  double *xzu = nullptr, *yzu = nullptr;  // z of each unique (x, z) / (y, z) key
  double *xu = nullptr, *yu = nullptr;
  int *ix = nullptr, *iy = nullptr;
  // plan-time sort scratch (index.hip): keys and focus numbers, ping-pong
  uint64_t *skey0 = nullptr, *skey1 = nullptr;
  int *sval0 = nullptr, *sval1 = nullptr, *shist = nullptr, *shead = nullptr, *srank = nullptr;
  int *rows = nullptr, *cols = nullptr, *row_pos = nullptr, *col_pos = nullptr;
  int *keep_row = nullptr, *keep_col = nullptr;
  float *aeff = nullptr;                 // [ny][nx] effective amplitude (user orientation)
  double *ucoord = nullptr, *vcoord = nullptr;
  int *csr_ptr = nullptr, *csr_foci = nullptr;
  int *csr_ic = nullptr;                 // reduced-grid column of the focus at each CSR position
  int *csr_ir = nullptr;                 // reduced-grid row of the focus at each CSR position
  int *scalars = nullptr;                // plan-time integer results
  double *dscalars = nullptr;            // plan-time float64 results
  double *ap_part = nullptr;             // aperture statistics, per workgroup
  int *ap_cnt = nullptr;
  int *dup = nullptr;
  // products and state (sized after the index work)
  float *omt_r = nullptr, *omt_i = nullptr, *omc_r = nullptr, *omc_i = nullptr;
  float *wc_r = nullptr, *wc_i = nullptr;
  float *amp = nullptr, *p_r = nullptr, *p_i = nullptr;
  float *s_r = nullptr, *s_i = nullptr;
  float *x_r = nullptr, *x_i = nullptr;  // operator-call scratch pupil
  float *theta = nullptr, *theta_new = nullptr;   // interleaved [2*nf]
  float *intensity = nullptr;            // [nf]
  double *w = nullptr, *stats = nullptr, *hist = nullptr;
  double *fixph = nullptr;               // [2 nf] frozen focal phasors (phase fixing)
  double *upd_s1 = nullptr, *upd_s2 = nullptr;   // many-focus update partials
  int *upd_snap = nullptr;
  int *ctrl = nullptr;
  float *iobuf = nullptr;                // [2*ny*nx] staging for operator calls
  float *part = nullptr;                 // split-K partial tiles (shared by both products)
  float *gpart = nullptr;                // fused-gather partials [tiles_n][ldp] complex
  // split-precision modes: 16-bit term planes [re/im][term] of a [row][K]
  // matrix each, stored k-blocked (kblk_index)
  unsigned short *as_f = nullptr;        // Omega_r            [2][NT] x [Urp][Rp]
  unsigned short *as_b = nullptr;        // Omega_r^H          [2][NT] x [Rp][Urp]
  unsigned short *ps = nullptr;          // pupil field P^T    [2][NT] x [Cp][Rp]
  unsigned short *ss = nullptr;          // scatter S^T        [2][NT] x [Cp][Urp]
  unsigned short *xs = nullptr;          // operator-call P^T  [2][NT] x [Cp][Rp]
  // adjoint re-associated when every reduced row holds one focus:
  // E' = (Omega_r^H diag Theta') conj(Omega_c rows of the foci)
  float *ob_r = nullptr, *ob_i = nullptr;   // Omega_r^H float32, as_b's layout [Rp][Urp]
  unsigned short *as_s = nullptr;        // Omega_r^H diag Theta' [2][NT] x [Rp][Urp]
  unsigned short *bs = nullptr;          // conj Omega_c rows      [2][NT] x [Cp][Urp]
  float *unit = nullptr;                 // [2 nf] unit focal values (plan time)
  // grid form (float32): the second product of Eq. 2 formed densely
  float *lt_r = nullptr, *lt_i = nullptr;   // L^T            [Cp][Urp]
  float *wt_r = nullptr, *wt_i = nullptr;   // Omega_c        [Cp][Ucp]
  float *wn_i = nullptr;                    // -Im Omega_c^T  [Ucp][Cp] (with wc_r: conj)
  float *g_r = nullptr, *g_i = nullptr;     // reduced grid   [Urp][Ucp]
  float *tg_r = nullptr, *tg_i = nullptr;   // new field on the grid, transposed [Ucp][Urp]
};

// Number of 16-bit terms per float32 operand of a precision mode (0: float32).
__host__ __device__ inline int split_terms_of(int precision) {
  return precision == GSWMTP_BF16X3 || precision == GSWMTP_FP16X3 ? 2
         : precision == GSWMTP_BF16X6                             ? 3
                                                                  : 0;
}
__host__ __device__ inline bool split_is_bf16(int precision) {
  return precision == GSWMTP_BF16X3 || precision == GSWMTP_BF16X6;
}

// Round-to-nearest-even float32 -> bfloat16 / float16 bit patterns and back.
__device__ __forceinline__ unsigned short f32_to_bf16_rn(float f) {
  // one v_cvt_pk_bf16_f32 (round to nearest even) on gfx950
  return __builtin_bit_cast(unsigned short, (__bf16)f);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float((unsigned)h << 16);
}
__device__ __forceinline__ unsigned short f32_to_f16_rn(float f) {
  return __builtin_bit_cast(unsigned short, (_Float16)f);
}
__device__ __forceinline__ float f16_to_f32(unsigned short h) {
  return (float)__builtin_bit_cast(_Float16, h);
}

// x = t0 + t1 (+ t2) in 16-bit terms: t0 = rn(x), t1 = rn(x - t0), ...; the
// float32 remainders are exact.  out[q * stride] receives term q.
template <bool BF, int NT>
__device__ __forceinline__ void split_terms(float x, unsigned short *out, int stride) {
  float r = x;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const unsigned short h = BF ? f32_to_bf16_rn(r) : f32_to_f16_rn(r);
    out[q * stride] = h;
    r = r - (BF ? bf16_to_f32(h) : f16_to_f32(h));
  }
}
__device__ __forceinline__ float join_terms(bool bf, int nt, const unsigned short *t,
                                            size_t stride) {
  float v = 0.f;
  for (int q = nt - 1; q >= 0; --q) v += bf ? bf16_to_f32(t[q * stride]) : f16_to_f32(t[q * stride]);
  return v;
}

// Phase-only projection of one back-propagated sample onto the amplitude
// constraint: A c / |c|, phasor 1 where c = 0, 0 outside the aperture.
__device__ __forceinline__ void project_amp(float cr, float ci, float am, float &pr, float &pi) {
  // one explicit fma, so every kernel that projects (the product epilogues
  // and the split-K tail kernels) rounds |c|^2 alike; left to the compiler,
  // the contraction may differ between kernels
  const float mag2 = fmaf(cr, cr, ci * ci);
  pr = 0.f;
  pi = 0.f;
  if (am > 0.f) {
    if (mag2 > 0.f) {
      const float sc = am * rsqrtf(mag2);
      pr = cr * sc;
      pi = ci * sc;
    } else {
      pr = am;
    }
  }
}

// Placement of the four waves of a product workgroup: 2 x 2 waves of
// BM/2 x BN/2 each, or (COLS, the loop that reads B straight into registers)
// 1 x 4 waves of BM x BN/4, so that no two waves share a B row.  MB x NB
// 32x32 MFMA blocks per wave; item r of lane (l32, h) of a block is row
// 8 (r/4) + 4 h + r % 4, column l32.
template <int BM, int BN, bool COLS = false>
struct WaveLayout {
  static constexpr int WTM = COLS ? BM : BM / 2, WTN = COLS ? BN / 4 : BN / 2;
  static constexpr int MB = WTM / 32, NB = WTN / 32;
  __device__ static int wm(int wave) { return COLS ? 0 : (wave & 1); }
  __device__ static int wn(int wave) { return COLS ? wave : (wave >> 1); }
};

// Position in the BM x BN tile of partial-sum slot (i, j, r) of thread tid.
template <int BM, int BN, bool COLS = false>
__device__ __forceinline__ void tile_slot_pos(int tid, int i, int j, int r, int &m, int &n) {
  using L = WaveLayout<BM, BN, COLS>;
  const int lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, h = lane >> 5;
  m = L::wm(wave) * L::WTM + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
  n = L::wn(wave) * L::WTN + j * 32 + l32;
}

// complex tile M x N, K per stage; split products: kg k-groups of four waves,
// pipe: 1 software-pipelined fragment reads (one k-group), 2 the same with
// the B operand read straight into registers (1 x 4 waves, two terms), 3 the
// 16x16-block loop (B straight into registers, BM a multiple of 16, no K
// split; adjoint epilogues only)
struct GemmTile { int bm = 64, bn = 64, bk = 16, kg = 1, pipe = 0; };

// Launch schedule of one complex product: t_dp whole tiles, then n_tail tiles
// split along K into `split` chunks (grid = t_dp + n_tail * split).
struct GemmSched {
  GemmTile tile;
  int tiles_m = 0, tiles = 0;
  int t_dp = 0, n_tail = 0, split = 1;
  int grid = 0;
  size_t part_floats = 0;
  int xgm = 1;                  // 16x16-block loop: XCD groups of M tiles
};

typedef float gsw_v16f __attribute__((ext_vector_type(16)));

// Where the fused focus gather reads and writes.
struct GatherCtx {
  float *part;                 // [tiles_n][ldp] interleaved complex partial sums
  const int *ptr;              // CSR row pointers over the reduced r rows [Ur + 1]
  const int *foci;             // foci sorted by (ir, ic)
  const int *ir, *ic;          // reduced-grid row / column of every focus
  const int *cir, *cic;        // the same at each CSR position (sorted foci)
  const float *wcr, *wci;      // Omega_c^T planes [Uc][Cp]
  int nf, Ur, Cp;
  int ldp;                     // foci per partial row (nf rounded up to even)
};

// Focus indices of a tile's gather, read ahead of the product's main loop so
// that the epilogue waits only for the Omega_c rows: the CSR range of the
// tile's reduced rows (first, with the operand loads), then lane l of every
// wave takes CSR position p0 + l (the tile's first 64 foci).
struct GatherPre {
  int p0 = 0, p1 = 0;       // CSR positions of the tile's reduced rows
  int f = 0, a = 0, c = 0;  // this lane's focus, its row in the tile, its column
  bool loaded = false;
};
__device__ __forceinline__ void gather_pre_rows(const GatherCtx &g, int m0, int bm,
                                                GatherPre &q) {
  const int r0 = m0 < g.Ur ? m0 : g.Ur, r1 = m0 + bm < g.Ur ? m0 + bm : g.Ur;
  q.p0 = g.ptr[r0];
  q.p1 = g.ptr[r1];
}
__device__ __forceinline__ void gather_pre_foci(const GatherCtx &g, int m0, int tid,
                                                GatherPre &q) {
  const int pp = q.p0 + (tid & 63);
  const bool ok = pp < q.p1;
  q.f = ok ? g.foci[pp] : 0;
  q.a = ok ? g.cir[pp] - m0 : 0;
  q.c = ok ? g.cic[pp] : 0;
  q.loaded = true;
}

// The focus gather of one BM x BN tile of L staged in LDS (real part at
// lds[m (BN + 1) + n], imaginary part BM (BN + 1) floats further on): the
// tile's foci are taken 64 at a time, one per lane: wave w forms
//   sum_{n in its BN/4 columns} L[ir][n] Wc[ic][n]
// for the lane's focus (its Omega_c run read as 16-byte loads, all in
// flight together), the four waves' sums are added in wave order and the
// result written as partial number prow of that focus (n0 / BN for a whole-K
// tile; the batched form's K chunks of a forward tile write partial rows of
// their own, which the focus update adds like the column tiles').
template <int BM, int BN>
__device__ __forceinline__ void gather_tile_lds(const GatherCtx &g, float *lds, int m0, int n0,
                                                int tid, const GatherPre &q, int prow) {
  constexpr int LD = BN + 1;
  constexpr int CW = BN / 4;   // columns per wave
  typedef float f4 __attribute__((ext_vector_type(4)));
  const int lane = tid & 63, wave = tid >> 6;
  float *tr = lds, *ti = lds + BM * LD;
  float *red = lds + 2 * BM * LD;   // [4 waves][64 lanes][re, im]
  const int p0 = q.p0, nfoc = q.p1 - q.p0;
  float *out = g.part + 2 * (size_t)prow * g.ldp;
  for (int u0 = 0; u0 < nfoc; u0 += 64) {
    const bool on = u0 + lane < nfoc;
    int f = q.f, a = q.a, c = q.c;
    if (u0 > 0) {
      const int pp = on ? p0 + u0 + lane : p0;
      f = g.foci[pp];
      a = g.cir[pp] - m0;
      c = g.cic[pp];
    }
    float sr = 0.f, si = 0.f;
    if (on) {
      const size_t wrow = (size_t)c * g.Cp + n0 + wave * CW;
      f4 wr[CW / 4], wi[CW / 4];
#pragma unroll
      for (int k = 0; k < CW / 4; ++k) {
        wr[k] = *reinterpret_cast<const f4 *>(g.wcr + wrow + 4 * k);
        wi[k] = *reinterpret_cast<const f4 *>(g.wci + wrow + 4 * k);
      }
      const float *lr = tr + a * LD + wave * CW, *li = ti + a * LD + wave * CW;
#pragma unroll
      for (int k = 0; k < CW / 4; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float xr = lr[4 * k + e], xi = li[4 * k + e];
          sr = fmaf(xr, wr[k][e], fmaf(-xi, wi[k][e], sr));
          si = fmaf(xr, wi[k][e], fmaf(xi, wr[k][e], si));
        }
    }
    red[2 * (wave * 64 + lane)] = sr;
    red[2 * (wave * 64 + lane) + 1] = si;
    __syncthreads();
    if (wave == 0 && on) {
      float tr_ = red[2 * lane], ti_ = red[2 * lane + 1];
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        tr_ += red[2 * (w * 64 + lane)];
        ti_ += red[2 * (w * 64 + lane) + 1];
      }
      out[2 * f] = tr_;
      out[2 * f + 1] = ti_;
    }
    __syncthreads();   // the sums are read before the next round writes them
  }
}

// Focus gather fused into the forward product's epilogue (the second
// product of Eq. 2, formed only at the foci).  The BM x BN complex tile of
// L = Omega_r P held in the accumulators is staged in LDS, then gathered by
// gather_tile_lds.  Accumulator item r of lane (l32, h) of a 32x32 block
// holds row 8 (r/4) + 4 h + r % 4, column l32.
template <int BM, int BN, bool COLS = false>
__device__ __forceinline__ void gather_epilogue(
    const GatherCtx &g,
    const gsw_v16f (&accR)[WaveLayout<BM, BN, COLS>::MB][WaveLayout<BM, BN, COLS>::NB],
    const gsw_v16f (&accI)[WaveLayout<BM, BN, COLS>::MB][WaveLayout<BM, BN, COLS>::NB],
    float *lds, int m0, int n0, int tid, GatherPre q, int prow = -1) {
  using L = WaveLayout<BM, BN, COLS>;
  constexpr int MB = L::MB, NB = L::NB, WTM = L::WTM, WTN = L::WTN, LD = BN + 1;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = L::wm(wave), wn = L::wn(wave), l32 = lane & 31, h = lane >> 5;
  float *tr = lds, *ti = lds + BM * LD;
  if (!q.loaded) {
    gather_pre_rows(g, m0, BM, q);
    gather_pre_foci(g, m0, tid, q);
  }
  __syncthreads();   // operand stages are no longer read
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ml = wm * WTM + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        const int nl = wn * WTN + j * 32 + l32;
        tr[ml * LD + nl] = accR[i][j][r];
        ti[ml * LD + nl] = accI[i][j][r];
      }
  __syncthreads();
  gather_tile_lds<BM, BN>(g, lds, m0, n0, tid, q, prow >= 0 ? prow : n0 / BN);
}

// The same without indices read ahead (they are read at the epilogue).
template <int BM, int BN, bool COLS = false>
__device__ __forceinline__ void gather_epilogue(
    const GatherCtx &g,
    const gsw_v16f (&accR)[WaveLayout<BM, BN, COLS>::MB][WaveLayout<BM, BN, COLS>::NB],
    const gsw_v16f (&accI)[WaveLayout<BM, BN, COLS>::MB][WaveLayout<BM, BN, COLS>::NB],
    float *lds, int m0, int n0, int tid, int prow = -1) {
  gather_epilogue<BM, BN, COLS>(g, accR, accI, lds, m0, n0, tid, GatherPre{}, prow);
}

template <int BM, int BN>
constexpr int gather_lds_bytes() { return 2 * BM * (BN + 1) * 4 + 4 * 64 * 2 * 4; }

}  // namespace gswmtp

struct gswmtp_plan {
  int device = 0;
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_user = nullptr, ev_int = nullptr;
  hipEvent_t ev_t[GSWMTP_N_STAGES + 1] = {};
  gswmtp::Dims d;
  gswmtp::Bufs b;
  int precision = GSWMTP_FP32;
  int weighting = GSWMTP_WEIGHT_GSW;
  gswmtp::GemmSched sched_fwd, sched_bwd;
  // grid form: first product transposed (L^T = P^T Omega_r^T), grid product
  // G = L Omega_c^T, and the scatter product S = Theta'_grid conj(Omega_c)
  bool grid_form = false;
  gswmtp::GemmSched sched_f1, sched_f2, sched_a1;
  // split modes with one focus in every reduced row: the adjoint's left
  // operand carries Theta' (no scatter; the right operand is fixed)
  bool scaled_adj = false;
  int cus = 256;
  int amp_exp = 0;                        // split modes: P carries amp * 2^amp_exp
  void *pool0 = nullptr, *pool1 = nullptr;
  size_t pool0_bytes = 0, pool1_bytes = 0;
  void *ws = nullptr;                     // caller's workspace holding both pools, or null
  size_t ws_bytes = 0;
  hipGraphExec_t graph1 = nullptr, graph8 = nullptr;
  bool fwd_valid = false;                 // theta and intensity match the current phase
  bool stats_valid = false;               // so do the focus statistics (implies fwd_valid)
  const double *meas_active = nullptr;    // b.meas while a measured pass is queued, else null
  bool use_graph = true;
  int fault_alloc = -1;                   // allocation fault injection (fault_alloc_setting)
  int n_alloc = 0;                        // device allocations made by the create call
  std::string err;
};

namespace gswmtp {

// Allocation fault injection for testing the failure paths, read from the
// environment at each create call: GSWMTP_FAULT_INJECT=alloc makes every
// device allocation of the call fail (the call returns GSWMTP_E_NOMEM before
// any device work), =alloc:K only its K-th one (K >= 1; the earlier ones
// succeed and are released by the failure path).  -1: off.
int fault_alloc_setting();
// Whether the device allocation about to be made - the (*count + 1)-th of
// the call - is the injected failure; advances *count.
bool fault_alloc_hit(int setting, int *count);

// Plan-time index work by sorting (index.hip).  IndexScratch holds two
// (key, focus number) buffers of n entries, the digit counts
// (index_hist_ints(n)) and the group heads and ranks (n each).
struct IndexScratch {
  uint64_t *key[2];
  int *val[2];
  int *hist, *head, *rank;
};
size_t index_hist_ints(int n);
// Distinct (coordinate, z) pairs of n foci in increasing order (coordinate,
// then z; -0.0 is +0.0): uniq / uniq_z receive them, idx[i] the position of
// focus i's pair among them, *count (device) their number.  has_z = false
// when every z is zero (one sort of the coordinates suffices).
hipError_t unique_pairs(const double *c, const double *z, bool has_z, int n, IndexScratch sc,
                        int *idx, double *uniq, double *uniq_z, int *count, hipStream_t s);
// Foci ordered by the index pair (hi, lo) (each < 2^18), ties in focus
// order: order[pos] = focus number (nullable); *dup (device, nullable) is
// or-ed with 1 when two foci share a pair.
hipError_t pair_order(const int *hi, const int *lo, int n, IndexScratch sc, int *order,
                      int *dup, hipStream_t s);

// Kernel launchers (stream-ordered, no synchronisation).
// honour_done: the kernel returns at once when the plan's done flag is set
// (early termination inside a queued / graph-replayed run of passes).
// phases: bit 0 the product launch, bit 1 the split-K tail launch (if any).
hipError_t launch_cgemm(const gswmtp_plan *p, bool forward, int epi, const float *br,
                        const float *bi, float *cr, float *ci, const float *er,
                        const float *ei, bool honour_done, hipStream_t s, int phases = 3);
hipError_t launch_gather_reduce(const gswmtp_plan *p, float *theta, float scale, hipStream_t s);
// Theta and |Theta|^2 of the current forward's gather partials into the
// plan's theta and intensity, and into field / intensity when not null (no
// statistics, one launch).
hipError_t launch_field(const gswmtp_plan *p, hipStream_t s, float *field = nullptr,
                        float *intensity = nullptr);
GatherCtx gather_ctx(const gswmtp_plan *p);
hipError_t launch_cgemm_split(const gswmtp_plan *p, bool forward, int epi,
                              const unsigned short *bt, float *cr, float *ci,
                              unsigned short *pt_out, bool honour_done, hipStream_t s,
                              int phases = 3, const unsigned short *at = nullptr);
// out: the S^T planes written (null: the plan's scatter buffer)
hipError_t launch_scatter_split(const gswmtp_plan *p, const float *theta_new, float scale,
                                bool honour_done, hipStream_t s, unsigned short *out = nullptr);
// Omega_r^H diag(Theta') as split planes (plans with scaled_adj)
hipError_t launch_scale_adjoint_split(const gswmtp_plan *p, bool honour_done, hipStream_t s);
hipError_t launch_update(const gswmtp_plan *p, int mode, hipStream_t s);
hipError_t launch_grad_field(const gswmtp_plan *p, const float *g, hipStream_t s);
hipError_t launch_scatter(const gswmtp_plan *p, const float *theta_new, bool honour_done,
                          hipStream_t s);
const char *cgemm_kernel_name(const gswmtp_plan *p, bool forward, int epi);
// A float32 complex product with explicit operands: C[M][N] = sum_k A[m][k] B[k][n]
// with A given k-major (AT[k][m], row pitch lda) and B row-major (pitch ldb).
hipError_t launch_cgemm_ex(const gswmtp_plan *p, const GemmSched &sc, const float *atr,
                           const float *ati, int lda, const float *br, const float *bi, int ldb,
                           float *cr, float *ci, int ldc, int M, int N, int K, int epi,
                           bool honour_done, hipStream_t s);
// A split product with explicit operands (16-bit term planes of [rows][K]
// matrices, k-blocked): C[M][N] = sum_k A[m][k] B[n][k] into float32 planes
// [M][ldc] on schedule sc.
hipError_t launch_cgemm_split_ex(const gswmtp_plan *p, const GemmSched &sc,
                                 const unsigned short *a, int M, const unsigned short *b, int N,
                                 int K, float *cr, float *ci, int ldc, bool honour_done,
                                 hipStream_t s);
// Split grid form: float32 S [Urp][Cp] (times scale) as the split planes of
// S^T in the plan's scatter buffer.
hipError_t launch_split_transpose(const gswmtp_plan *p, const float *sr, const float *si,
                                  float scale, bool honour_done, hipStream_t s);
// Grid form: Theta_n = G[ir_n][ic_n] into the gather partials (one per focus);
// Theta'_n (times g_n when g is not null) onto the transposed grid at
// (ic_n, ir_n).
hipError_t launch_grid_gather(const gswmtp_plan *p, hipStream_t s);
hipError_t launch_grid_scatter(const gswmtp_plan *p, const float *theta_new, float scale,
                               hipStream_t s, const float *g = nullptr);
// Gather partials per focus of the plan's forward form.
int gather_partials(const gswmtp_plan *p);
int gather_ld(const gswmtp_plan *p);   // gather partial row stride: nf rounded up to even
// min_chunk_div > 0: at most that many K chunks per tail tile, so each keeps
// at least KT / min_chunk_div stages (and never fewer than two).
GemmSched make_sched(int M, int N, int K, GemmTile tile, int cus, bool allow_split,
                     int min_chunk_div = 0);

// One unit of a batched product's device work list: tile `tile` of item
// `item` (a plan's product arguments), K stages [kb, ke), its focus-gather
// partials (forward) written to partial row `prow`.
struct WorkUnit {
  int item, tile, kb, ke, prow, pad0, pad1, pad2;
};
// Kernel configuration of a batched product: tile, loop (GemmTile::pipe;
// k-groups for the three-term split) and the forward's K chunks per tile.
struct WorkConfig {
  GemmTile tile;
  int split = 1;
  bool operator==(const WorkConfig &o) const {
    return tile.bm == o.tile.bm && tile.bn == o.tile.bn && tile.bk == o.tile.bk &&
           tile.kg == o.tile.kg && tile.pipe == o.tile.pipe && split == o.split;
  }
};
// Persistent (or one-unit-per-workgroup) launch over a work list of one
// configuration: workgroup b runs units d_off[b] .. d_off[b + 1] - 1, or
// unit b when d_off is null (grid = n_work).  Configurations with two
// k-groups always run one unit per workgroup.
struct WorkLaunch {
  WorkConfig cfg;
  int epi = 0, precision = 0;
  const void *d_items = nullptr;   // per-plan product arguments (CgemmArgs / SplitArgs)
  const WorkUnit *d_work = nullptr;
  const int *d_off = nullptr;      // [grid + 1] unit ranges per workgroup, or null
  int n_work = 0, grid = 0;
};
hipError_t launch_cgemm_work(const WorkLaunch &w, hipStream_t s);
hipError_t launch_cgemm_split_work(const WorkLaunch &w, hipStream_t s);
// Resident workgroups per CU of a configuration's work-list kernel (0: the
// configuration has no such kernel).
int cgemm_work_occupancy(const WorkConfig &c, int epi);
int cgemm_split_work_occupancy(const WorkConfig &c, int epi, int precision);

// Per-plan product arguments of the batched form for a work-list launch with
// tile (bm, bn) / `tl`: size of one item, and the tile count it fills in.
// honour_done: return at once when the plan's done flag is set.  cr / ci
// (float32 adjoint) and pt_out (split adjoint), nullable: write the
// projected field there instead of the plan's pupil field (tuning runs).
size_t cgemm_args_bytes();
int fill_cgemm_args(const gswmtp_plan *p, bool forward, int bm, int bn, bool honour_done,
                    float *cr, float *ci, void *out);
size_t split_args_bytes();
int fill_split_args(const gswmtp_plan *p, bool forward, const GemmTile &tl, bool honour_done,
                    unsigned short *pt_out, void *out);
// Split-precision scatter of the batched form.
size_t scatter_split_args_bytes();
int fill_scatter_split_args(const gswmtp_plan *p, void *out);
hipError_t launch_scatter_split_grouped(const void *items, const int *starts, int n, int blocks,
                                        int precision, hipStream_t s);
// Focus update: one workgroup of kUpdThreads holds up to kUpdRegFociMax foci
// in registers; more foci take the three-launch form over
// update_workgroups(nf) workgroups.
constexpr int kUpdThreads = 512;
constexpr int kUpdRegFociMax = 2 * kUpdThreads;
inline int update_workgroups(int nf) {
  return nf <= kUpdRegFociMax ? 0 : (nf + kUpdThreads - 1) / kUpdThreads;
}
struct GroupedUpdate {
  void *d_items = nullptr;     // every plan, phase-1 launch
  int *d_starts = nullptr;
  int n_items = 0, blocks = 0;
  void *d_big = nullptr;       // many-focus plans, phase-2 and -3 launches
  int *d_big_starts = nullptr;
  int n_big = 0, big_blocks = 0;
};
size_t update_args_bytes();
// Returns the plan's many-focus workgroup count (0: register form, one block).
// partials: gather partials per focus of the batch's forward product
int fill_update_args(const gswmtp_plan *p, int mode, int partials, void *out);
hipError_t launch_update_grouped(const GroupedUpdate &g, hipStream_t s);
size_t scatter_args_bytes();
int fill_scatter_args(const gswmtp_plan *p, void *out);
hipError_t launch_scatter_grouped(const void *d_items, const int *d_starts, int n, int blocks,
                                  hipStream_t s);

// Product epilogues: store C; project onto the amplitude constraint; phase
// gradient; focus gather (forward product only, C never stored).
enum { EPI_STORE = 0, EPI_PROJECT = 1, EPI_GRAD = 2, EPI_GATHER = 3 };
enum { UPD_ITERATE = 0, UPD_STATS = 1, UPD_GRAD = 2 };

}  // namespace gswmtp
