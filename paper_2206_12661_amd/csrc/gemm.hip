// Dense complex products of the matrix triple product (Eq. 2) on CDNA4 MFMA.
//
// Both products of a GSW pass have the same form
//     C[M][N] = sum_k A[m][k] B[k][n]          (complex, float32 planes)
// with A supplied k-major (AT[k][m]) and B row-major:
//   forward   L = Omega_r P       A^T = OmT [Rp][Urp], B = P [Rp][Cp]
//   adjoint   E' = Omega_r^H S    A^T = OmC [Urp][Rp], B = S [Urp][Cp]
// Every dimension is padded with zeros to a tile multiple, so the kernels
// have no bounds checks.
//
// Complex arithmetic uses four real products per complex product
// (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br) on v_mfma_f32_32x32x2_f32:
// 64 lanes, one float of A and one of B per lane, a 32x32 float32 block
// accumulated over K = 2 per instruction.  A workgroup of four waves owns a
// BM x BN complex tile; each wave a (BM/2) x (BN/2) quadrant.  K advances in
// stages of 16 complex values staged through LDS with double buffering, a
// register prefetch of the next stage from global memory and a one-step-ahead
// prefetch of the MFMA operands from LDS.
//
// Scheduling (256 CUs): full tiles are processed one workgroup each; when
// the tile count leaves a short last round, those tail tiles are split along
// K into `split` chunks so every CU gets about the same work.  Chunk partial
// sums go to a workspace; a second launch over the tail tiles adds each
// tile's chunks in fixed order and runs the epilogue (the launch boundary
// orders the workspace writes; no inter-workgroup fences or atomics).
//
// Epilogues: store C; project onto the amplitude constraint
// (E = A C / |C|, phasor 1 where C = 0: the phase-only projection of
// Algorithm 1, fused so E' never reaches HBM); or the phase gradient
// 2 Im(conj(E) C).
#include <cstring>

#include "gswmtp_internal.h"

namespace gswmtp {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));

struct CgemmArgs {
  const float *__restrict__ atr;
  const float *__restrict__ ati;
  const float *__restrict__ br;
  const float *__restrict__ bi;
  float *cr;
  float *ci;
  const float *__restrict__ amp;   // EPI_PROJECT: amplitude [M][ldc]
  const float *__restrict__ er;    // EPI_GRAD: pupil field planes [M][ldc]
  const float *__restrict__ ei;
  const int *done;                 // nullable: skip when *done != 0
  float *part;                     // split-K partial tiles
  GatherCtx g;                     // EPI_GATHER
  int phase;                       // 0: whole tiles and K chunks; 1: reduce chunks of tail tiles
  int lda, ldb, ldc;
  int M, N, K;
  int tiles_m;
  int t_dp;                        // tiles processed whole
  int split;                       // K chunks per tail tile
};

constexpr int kBK = 16;            // complex k per LDS stage
constexpr int kThreads = 256;

// Remap the hardware workgroup id so that the tiles each XCD (dispatched
// round-robin, id % 8) works on are contiguous in M-fastest tile order and
// share B column panels in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int bid, int tiles) {
  const int xcd = bid & 7, local = bid >> 3;
  const int per = tiles >> 3, rem = tiles & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

template <int MB, int NB, int EPI>
__device__ __forceinline__ void epilogue(const CgemmArgs &a, v16f (&accR)[MB][NB],
                                         v16f (&accI)[MB][NB], int mw, int nw, int l32,
                                         int h) {
  // Accumulator layout of the 32x32 f32 block: lane (l32, h), item r holds
  // row 8 (r / 4) + 4 h + r % 4, column l32.
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = mw + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        const int n = nw + j * 32 + l32;
        const size_t o = (size_t)m * a.ldc + n;
        const float cr = accR[i][j][r], ci = accI[i][j][r];
        if constexpr (EPI == EPI_STORE) {
          a.cr[o] = cr;
          a.ci[o] = ci;
        } else if constexpr (EPI == EPI_PROJECT) {
          float pr, pi;
          project_amp(cr, ci, a.amp[o], pr, pi);
          a.cr[o] = pr;
          a.ci[o] = pi;
        } else {
          a.cr[o] = 2.f * (a.er[o] * ci - a.ei[o] * cr);
        }
      }
}

template <int BM, int BN, int EPI>
constexpr int f32_lds_floats() {
  constexpr int A_F = 2 * 2 * kBK * (BM + 32), B_F = 2 * 2 * kBK * (BN + 32);
  constexpr int G_F = EPI == EPI_GATHER ? gather_lds_bytes<BM, BN>() / 4 : 0;
  return A_F + B_F > G_F ? A_F + B_F : G_F;
}

// One unit of a product: tile t over K stages [kb, ke).  tail < 0: the
// epilogue runs on the sums (a forward tile's gather writes partial row prow,
// -1: n0 / BN); tail >= 0 in phase 0: chunk `chunk` of tail tile `tail`
// stores its partial tile; phase 1 (kb = ke): tail tile `tail` adds its
// chunks' partials in order and runs the epilogue.
template <int BM, int BN, int EPI>
__device__ __forceinline__ void cgemm_f32_unit(const CgemmArgs &a, const int t, const int kb,
                                               const int ke, const int tail, const int chunk,
                                               const int prow, float *lds) {
  constexpr int WTM = BM / 2, WTN = BN / 2;    // wave tile (complex)
  constexpr int MB = WTM / 32, NB = WTN / 32;  // 32x32 blocks per wave
  constexpr int SA = BM + 32, SB = BN + 32;    // padded LDS row pitch (floats)
  constexpr int A4 = kBK * BM / 4;             // float4 per A plane per stage
  constexpr int B4 = kBK * BN / 4;
  constexpr int NA = 2 * A4 / kThreads, NBL = 2 * B4 / kThreads;
  static_assert(2 * A4 % kThreads == 0 && 2 * B4 % kThreads == 0, "tile/thread mismatch");

  // operand stages [buf][plane][k][row]; the gather epilogue reuses the space
  constexpr int A_F = 2 * 2 * kBK * SA;
  float *const sA = lds;
  float *const sB = lds + A_F;
  constexpr int BUF_A = 2 * kBK * SA, BUF_B = 2 * kBK * SB;

  const int tid = threadIdx.x;
  const int m0 = (t % a.tiles_m) * BM;
  const int n0 = (t / a.tiles_m) * BN;

  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int l32 = lane & 31, h = lane >> 5;

  v16f accR[MB][NB], accI[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      accR[i][j] = v16f{0};
      accI[i][j] = v16f{0};
    }

  // Staging map: float4 s of this thread covers plane idx / A4 of the tile,
  // row k = (idx % A4) / (BM / 4), columns 4 m4 .. 4 m4 + 3.
  v4f ra[NA], rb[NBL];
  const float *ga[NA];
  const float *gb[NBL];
  int la[NA], lb[NBL];
#pragma unroll
  for (int s = 0; s < NA; ++s) {
    const int idx = tid + kThreads * s;
    const int plane = idx / A4, rem = idx % A4;
    const int k = rem / (BM / 4), m4 = rem % (BM / 4);
    ga[s] = (plane ? a.ati : a.atr) + (size_t)k * a.lda + m0 + 4 * m4;
    la[s] = plane * (kBK * SA) + k * SA + 4 * m4;
  }
#pragma unroll
  for (int s = 0; s < NBL; ++s) {
    const int idx = tid + kThreads * s;
    const int plane = idx / B4, rem = idx % B4;
    const int k = rem / (BN / 4), n4 = rem % (BN / 4);
    gb[s] = (plane ? a.bi : a.br) + (size_t)k * a.ldb + n0 + 4 * n4;
    lb[s] = plane * (kBK * SB) + k * SB + 4 * n4;
  }
  const size_t stepA = (size_t)kBK * a.lda, stepB = (size_t)kBK * a.ldb;

  if (kb < ke) {
#pragma unroll
    for (int s = 0; s < NA; ++s)
      ra[s] = *reinterpret_cast<const v4f *>(ga[s] + (size_t)kb * stepA);
#pragma unroll
    for (int s = 0; s < NBL; ++s)
      rb[s] = *reinterpret_cast<const v4f *>(gb[s] + (size_t)kb * stepB);
  }
  // The done flag is read while the first stage is in flight (the loads are
  // kept above the test), not before it.
  const int stop = a.done ? *a.done : 0;
  asm volatile("" ::: "memory");
  if (stop) return;
  if (kb < ke) {
#pragma unroll
    for (int s = 0; s < NA; ++s) *reinterpret_cast<v4f *>(&sA[la[s]]) = ra[s];
#pragma unroll
    for (int s = 0; s < NBL; ++s) *reinterpret_cast<v4f *>(&sB[lb[s]]) = rb[s];
  }
  __syncthreads();
  for (int kt = kb; kt < ke; ++kt) {
    const int buf = (kt - kb) & 1;
    const bool more = kt + 1 < ke;
    if (more) {
#pragma unroll
      for (int s = 0; s < NA; ++s)
        ra[s] = *reinterpret_cast<const v4f *>(ga[s] + (size_t)(kt + 1) * stepA);
#pragma unroll
      for (int s = 0; s < NBL; ++s)
        rb[s] = *reinterpret_cast<const v4f *>(gb[s] + (size_t)(kt + 1) * stepB);
    }
    const float *pa = sA + buf * BUF_A + wm * WTM + l32;
    const float *pb = sB + buf * BUF_B + wn * WTN + l32;
    // MFMA operands of k pair p sit in slot p & 1; the next pair's operands
    // are read from LDS while the current pair's MFMAs run.  Lanes 0-31 take
    // k = 2p, lanes 32-63 take k = 2p + 1.
    float ar[2][MB], ai[2][MB], br[2][NB], bi[2][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      ar[0][i] = pa[h * SA + i * 32];
      ai[0][i] = pa[kBK * SA + h * SA + i * 32];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      br[0][j] = pb[h * SB + j * 32];
      bi[0][j] = pb[kBK * SB + h * SB + j * 32];
    }
#pragma unroll
    for (int p = 0; p < kBK / 2; ++p) {
      const int c = p & 1, q = c ^ 1;
      if (p + 1 < kBK / 2) {
        const int k = 2 * (p + 1) + h;
#pragma unroll
        for (int i = 0; i < MB; ++i) {
          ar[q][i] = pa[k * SA + i * 32];
          ai[q][i] = pa[kBK * SA + k * SA + i * 32];
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          br[q][j] = pb[k * SB + j * 32];
          bi[q][j] = pb[kBK * SB + k * SB + j * 32];
        }
      }
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          accR[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[c][i], br[c][j], accR[i][j], 0, 0, 0);
          accR[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai[c][i], bi[c][j], accR[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[c][i], bi[c][j], accI[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[c][i], br[c][j], accI[i][j], 0, 0, 0);
        }
    }
    if (more) {
      float *qa = sA + (buf ^ 1) * BUF_A;
      float *qb = sB + (buf ^ 1) * BUF_B;
#pragma unroll
      for (int s = 0; s < NA; ++s) *reinterpret_cast<v4f *>(&qa[la[s]]) = ra[s];
#pragma unroll
      for (int s = 0; s < NBL; ++s) *reinterpret_cast<v4f *>(&qb[lb[s]]) = rb[s];
    }
    __syncthreads();
  }

  constexpr int unit = 2 * MB * NB * 16 * kThreads;
  if (a.phase == 0 && tail >= 0) {
    // Partial tile of one K chunk in a thread-major layout (each store
    // instruction writes one float per lane, contiguous across lanes).
    float *pu = a.part + (size_t)(tail * a.split + chunk) * unit + tid;
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int o = (((i * NB + j) * 16 + r) * 2) * kThreads;
          pu[o] = accR[i][j][r];
          pu[o + kThreads] = accI[i][j][r];
        }
    return;
  }
  if (a.phase == 1) {
    // sum the tile's chunks in chunk order
    const float *pt = a.part + (size_t)tail * a.split * unit + tid;
    for (int c = 0; c < a.split; ++c) {
      const float *pc = pt + (size_t)c * unit;
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int o = (((i * NB + j) * 16 + r) * 2) * kThreads;
            accR[i][j][r] += pc[o];
            accI[i][j][r] += pc[o + kThreads];
          }
    }
  }
  if constexpr (EPI == EPI_GATHER)
    gather_epilogue<BM, BN>(a.g, accR, accI, lds, m0, n0, tid, prow);
  else
    epilogue<MB, NB, EPI>(a, accR, accI, m0 + wm * WTM, n0 + wn * WTN, l32, h);
}

// One workgroup's share of a product: whole tile, K chunk (phase 0) or tail
// reduction (phase 1) number `bid` of the schedule in `a`.
template <int BM, int BN, int EPI>
__device__ __forceinline__ void cgemm_f32_body(const CgemmArgs &a, const int bid, float *lds) {
  const int KT = a.K / kBK;
  if (a.phase == 1) {
    cgemm_f32_unit<BM, BN, EPI>(a, a.t_dp + bid, 0, 0, bid, 0, -1, lds);
  } else if (bid < a.t_dp) {
    cgemm_f32_unit<BM, BN, EPI>(a, xcd_tile(bid, a.t_dp), 0, KT, -1, 0, -1, lds);
  } else {
    const int u = bid - a.t_dp, tail = u / a.split, chunk = u % a.split;
    cgemm_f32_unit<BM, BN, EPI>(a, a.t_dp + tail, chunk * KT / a.split,
                                (chunk + 1) * KT / a.split, tail, chunk, -1, lds);
  }
}

// Work-list launch (batched form): workgroup b runs the units off[b] ..
// off[b + 1] - 1 of the list (a persistent grid, the ranges balanced on the
// host), or unit b alone when off is null; each unit is a tile (or the K
// chunk of a forward tile) of one plan's product; the LDS is reused from unit
// to unit behind a barrier.
template <int BM, int BN, int EPI>
__global__ __launch_bounds__(kThreads) void cgemm_f32_work(const CgemmArgs *items,
                                                           const WorkUnit *work, const int *off, int n) {
  __shared__ __attribute__((aligned(16))) float lds[f32_lds_floats<BM, BN, EPI>()];
  // units off[b] .. off[b + 1] - 1 (persistent), or unit b (off null)
  const int w0 = off ? off[blockIdx.x] : (int)blockIdx.x;
  const int w1 = off ? off[blockIdx.x + 1] : w0 + 1;
  for (int w = w0; w < w1 && w < n; ++w) {
    if (w != w0) __syncthreads();   // the previous unit's LDS reads are done
    const WorkUnit u = work[w];
    cgemm_f32_unit<BM, BN, EPI>(items[u.item], u.tile, u.kb, u.ke, -1, 0, u.prow, lds);
  }
}

template <int BM, int BN, int EPI>
__global__ __launch_bounds__(kThreads) void cgemm_f32_mfma(CgemmArgs a) {
  __shared__ __attribute__((aligned(16))) float lds[f32_lds_floats<BM, BN, EPI>()];
  cgemm_f32_body<BM, BN, EPI>(a, blockIdx.x, lds);
}

// Split-K tail with the projection epilogue: adds the K-chunk partials of
// each tail tile in chunk order (the sums the product's own reduction
// launch would form) and projects, with many workgroups per tile so the
// partial reads are spread over the chip.  Block (tail, g) covers slots
// r = 4g .. 4g + 3 of every (i, j) block of the tile.
template <int BM, int BN>
__global__ __launch_bounds__(kThreads) void cgemm_tail_project(CgemmArgs a) {
  constexpr int MB = BM / 64, NB = BN / 64;
  constexpr int unit = 2 * MB * NB * 16 * kThreads;
  const int tail = blockIdx.x, g = blockIdx.y, tid = threadIdx.x;
  const int t = a.t_dp + tail;
  const int m0 = (t % a.tiles_m) * BM, n0 = (t / a.tiles_m) * BN;
  const float *pt = a.part + (size_t)tail * a.split * unit + tid;
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      size_t oc[4];
      float av[4];   // amplitudes read with the partials, not after them
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int m, n;
        tile_slot_pos<BM, BN>(tid, i, j, 4 * g + q, m, n);
        oc[q] = (size_t)(m0 + m) * a.ldc + n0 + n;
        av[q] = a.amp[oc[q]];
      }
      float sr[4] = {0.f, 0.f, 0.f, 0.f}, si[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
      for (int c = 0; c < a.split; ++c) {
        const float *pc = pt + (size_t)c * unit;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int o = (((i * NB + j) * 16 + 4 * g + q) * 2) * kThreads;
          sr[q] += pc[o];
          si[q] += pc[o + kThreads];
        }
      }
      if (a.done && *a.done) return;   // read after the partial sums
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float pr, pi;
        project_amp(sr[q], si[q], av[q], pr, pi);
        a.cr[oc[q]] = pr;
        a.ci[oc[q]] = pi;
      }
    }
}

template <int BM, int BN, int EPI>
hipError_t launch_t(const CgemmArgs &args, int grid, hipStream_t s) {
  hipLaunchKernelGGL((cgemm_f32_mfma<BM, BN, EPI>), dim3(grid), dim3(kThreads), 0, s, args);
  return hipGetLastError();
}

template <int EPI>
hipError_t launch_e(int bm, int bn, const CgemmArgs &args, int grid, hipStream_t s) {
  if (bm == 64 && bn == 64) return launch_t<64, 64, EPI>(args, grid, s);
  if (bm == 64 && bn == 128) return launch_t<64, 128, EPI>(args, grid, s);
  if (bm == 128 && bn == 64) return launch_t<128, 64, EPI>(args, grid, s);
  if (bm == 128 && bn == 128) return launch_t<128, 128, EPI>(args, grid, s);
  return hipErrorInvalidValue;
}

}  // namespace

GatherCtx gather_ctx(const gswmtp_plan *p) {
  GatherCtx g;
  g.part = p->b.gpart;
  g.ptr = p->b.csr_ptr;
  g.foci = p->b.csr_foci;
  g.ir = p->d.axis == 0 ? p->b.iy : p->b.ix;
  g.ic = p->d.axis == 0 ? p->b.ix : p->b.iy;
  g.cir = p->b.csr_ir;
  g.cic = p->b.csr_ic;
  g.wcr = p->b.wc_r;
  g.wci = p->b.wc_i;
  g.nf = p->d.nf;
  g.Ur = p->d.Ur;
  g.Cp = p->d.Cp;
  g.ldp = gather_ld(p);
  return g;
}

GemmSched make_sched(int M, int N, int K, GemmTile tile, int cus, bool allow_split,
                     int min_chunk_div) {
  GemmSched s;
  s.tile = tile;
  s.tiles_m = M / tile.bm;
  s.tiles = s.tiles_m * (N / tile.bn);
  const int KT = K / tile.bk;
  const int q = s.tiles / cus, r = s.tiles % cus;
  s.t_dp = s.tiles;
  s.n_tail = 0;
  s.split = 1;
  // Split the last round when it would leave more than a quarter of the CUs
  // idle; each chunk keeps at least two K stages and KT / min_chunk_div.
  if (allow_split && r > 0 && r * 4 < cus * 3 && KT >= 4) {
    int split = cus / r;
    if (split > KT / 2) split = KT / 2;
    if (min_chunk_div > 0 && split > min_chunk_div) split = min_chunk_div;
    if (split >= 2) {
      s.t_dp = q * cus;
      s.n_tail = r;
      s.split = split;
    }
  }
  s.grid = s.t_dp + s.n_tail * s.split;
  s.part_floats = (size_t)s.n_tail * s.split * tile.bm * tile.bn * 2;
  return s;
}

hipError_t launch_cgemm(const gswmtp_plan *p, bool forward, int epi, const float *br,
                        const float *bi, float *cr, float *ci, const float *er,
                        const float *ei, bool honour_done, hipStream_t s, int phases) {
  const Dims &d = p->d;
  const GemmSched &sc = forward ? p->sched_fwd : p->sched_bwd;
  CgemmArgs a{};
  if (forward) {
    a.atr = p->b.omt_r; a.ati = p->b.omt_i; a.lda = d.Urp;
    a.M = d.Urp; a.K = d.Rp;
  } else {
    a.atr = p->b.omc_r; a.ati = p->b.omc_i; a.lda = d.Rp;
    a.M = d.Rp; a.K = d.Urp;
  }
  a.br = br; a.bi = bi; a.ldb = d.Cp;
  a.cr = cr; a.ci = ci; a.ldc = d.Cp;
  a.N = d.Cp;
  a.amp = p->b.amp;
  a.er = er; a.ei = ei;
  a.done = honour_done ? p->b.ctrl + CTRL_DONE : nullptr;
  a.part = p->b.part;
  a.g = gather_ctx(p);
  if (epi == EPI_GATHER && !forward) return hipErrorInvalidValue;
  if (a.M % sc.tile.bm || a.N % sc.tile.bn || a.K % kBK) return hipErrorInvalidValue;
  if (sc.tiles_m * sc.tile.bm != a.M || sc.tiles * sc.tile.bm * sc.tile.bn != a.M * a.N)
    return hipErrorInvalidValue;
  a.tiles_m = sc.tiles_m;
  a.t_dp = sc.t_dp;
  a.split = sc.split;
  for (int phase = 0; phase < (sc.n_tail > 0 ? 2 : 1); ++phase) {
    if (!(phases & (1 << phase))) continue;
    a.phase = phase;
    const int grid = phase == 0 ? sc.grid : sc.n_tail;
    hipError_t e = hipErrorInvalidValue;
    if (phase == 1 && epi == EPI_PROJECT) {
      const dim3 tg(sc.n_tail, 4);
#define TAIL(BM, BN) hipLaunchKernelGGL((cgemm_tail_project<BM, BN>), tg, dim3(kThreads), 0, s, a)
      if (sc.tile.bm == 64 && sc.tile.bn == 64) TAIL(64, 64);
      else if (sc.tile.bm == 64 && sc.tile.bn == 128) TAIL(64, 128);
      else if (sc.tile.bm == 128 && sc.tile.bn == 64) TAIL(128, 64);
      else if (sc.tile.bm == 128 && sc.tile.bn == 128) TAIL(128, 128);
      else return hipErrorInvalidValue;
#undef TAIL
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      continue;
    }
    switch (epi) {
      case EPI_STORE: e = launch_e<EPI_STORE>(sc.tile.bm, sc.tile.bn, a, grid, s); break;
      case EPI_PROJECT: e = launch_e<EPI_PROJECT>(sc.tile.bm, sc.tile.bn, a, grid, s); break;
      case EPI_GRAD: e = launch_e<EPI_GRAD>(sc.tile.bm, sc.tile.bn, a, grid, s); break;
      case EPI_GATHER: e = launch_e<EPI_GATHER>(sc.tile.bm, sc.tile.bn, a, grid, s); break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cgemm_ex(const gswmtp_plan *p, const GemmSched &sc, const float *atr,
                           const float *ati, int lda, const float *br, const float *bi, int ldb,
                           float *cr, float *ci, int ldc, int M, int N, int K, int epi,
                           bool honour_done, hipStream_t s) {
  if (epi != EPI_STORE) return hipErrorInvalidValue;
  if (M % sc.tile.bm || N % sc.tile.bn || K % kBK) return hipErrorInvalidValue;
  if (sc.tiles_m * sc.tile.bm != M || sc.tiles * sc.tile.bm * sc.tile.bn != M * N)
    return hipErrorInvalidValue;
  CgemmArgs a{};
  a.atr = atr; a.ati = ati; a.lda = lda;
  a.br = br; a.bi = bi; a.ldb = ldb;
  a.cr = cr; a.ci = ci; a.ldc = ldc;
  a.M = M; a.N = N; a.K = K;
  a.done = honour_done ? p->b.ctrl + CTRL_DONE : nullptr;
  a.part = p->b.part;
  a.tiles_m = sc.tiles_m;
  a.t_dp = sc.t_dp;
  a.split = sc.split;
  for (int phase = 0; phase < (sc.n_tail > 0 ? 2 : 1); ++phase) {
    a.phase = phase;
    const hipError_t e = launch_e<EPI_STORE>(sc.tile.bm, sc.tile.bn, a,
                                             phase == 0 ? sc.grid : sc.n_tail, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

size_t cgemm_args_bytes() { return sizeof(CgemmArgs); }

// Arguments of plan p's product for a batched work-list launch with tile
// (bm, bn); the work units pick the tiles and K ranges.  honour_done: return at once when
// the plan's done flag is set.  cr / ci (adjoint only, nullable): write the
// projected field there instead of the plan's pupil field.  Returns the
// block count (tiles).
int fill_cgemm_args(const gswmtp_plan *p, bool forward, int bm, int bn, bool honour_done,
                    float *cr, float *ci, void *out) {
  const Dims &d = p->d;
  CgemmArgs a{};
  if (forward) {
    a.atr = p->b.omt_r; a.ati = p->b.omt_i; a.lda = d.Urp;
    a.M = d.Urp; a.K = d.Rp;
    a.br = p->b.p_r; a.bi = p->b.p_i;
  } else {
    a.atr = p->b.omc_r; a.ati = p->b.omc_i; a.lda = d.Rp;
    a.M = d.Rp; a.K = d.Urp;
    a.br = p->b.s_r; a.bi = p->b.s_i;
    a.cr = cr ? cr : p->b.p_r;
    a.ci = ci ? ci : p->b.p_i;
  }
  a.ldb = d.Cp;
  a.ldc = d.Cp;
  a.N = d.Cp;
  a.amp = p->b.amp;
  a.done = honour_done ? p->b.ctrl + CTRL_DONE : nullptr;
  a.part = p->b.part;
  a.g = gather_ctx(p);
  a.tiles_m = a.M / bm;
  a.t_dp = a.tiles_m * (a.N / bn);
  a.split = 1;
  a.phase = 0;
  std::memcpy(out, &a, sizeof a);
  return a.t_dp;
}

hipError_t launch_cgemm_work(const WorkLaunch &w, hipStream_t s) {
  if (w.n_work == 0) return hipSuccess;
  const auto *items = static_cast<const CgemmArgs *>(w.d_items);
  const GemmTile &t = w.cfg.tile;
#define WORK(BM, BN, EPI)                                                                   \
  hipLaunchKernelGGL((cgemm_f32_work<BM, BN, EPI>), dim3(w.grid), dim3(kThreads), 0, s, items, \
                     w.d_work, w.d_off, w.n_work)
#define WORK_EPI(BM, BN)                                        \
  do {                                                          \
    if (w.epi == EPI_GATHER) WORK(BM, BN, EPI_GATHER);          \
    else if (w.epi == EPI_PROJECT) WORK(BM, BN, EPI_PROJECT);   \
    else return hipErrorInvalidValue;                           \
  } while (0)
  if (t.bm == 64 && t.bn == 64) WORK_EPI(64, 64);
  else if (t.bm == 64 && t.bn == 128) WORK_EPI(64, 128);
  else if (t.bm == 128 && t.bn == 64) WORK_EPI(128, 64);
  else if (t.bm == 128 && t.bn == 128) WORK_EPI(128, 128);
  else return hipErrorInvalidValue;
#undef WORK_EPI
#undef WORK
  return hipGetLastError();
}

int cgemm_work_occupancy(const WorkConfig &c, int epi) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
#define OCC(BM, BN, EPI) \
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cgemm_f32_work<BM, BN, EPI>, kThreads, 0)
#define OCC_EPI(BM, BN)                                        \
  do {                                                         \
    if (epi == EPI_GATHER) OCC(BM, BN, EPI_GATHER);            \
    else if (epi == EPI_PROJECT) OCC(BM, BN, EPI_PROJECT);     \
  } while (0)
  const GemmTile &t = c.tile;
  if (t.bm == 64 && t.bn == 64) OCC_EPI(64, 64);
  else if (t.bm == 64 && t.bn == 128) OCC_EPI(64, 128);
  else if (t.bm == 128 && t.bn == 64) OCC_EPI(128, 64);
  else if (t.bm == 128 && t.bn == 128) OCC_EPI(128, 128);
#undef OCC_EPI
#undef OCC
  return e == hipSuccess ? n : 0;
}

const char *cgemm_kernel_name(const gswmtp_plan *p, bool forward, int) {
  if (!split_terms_of(p->precision)) return "cgemm_f32_mfma";
  const GemmSched &sc = forward ? p->sched_fwd : p->sched_bwd;
  return sc.tile.pipe == 3 ? "cgemm_split_d16" : "cgemm_split_mfma";
}

}  // namespace gswmtp
