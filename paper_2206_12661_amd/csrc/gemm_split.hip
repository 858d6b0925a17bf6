// Split-precision complex products of the matrix triple product (Eq. 2) on
// the CDNA4 16-bit matrix cores (v_mfma_f32_32x32x16_{bf16,f16}).
//
// Every float32 operand x is carried as NT 16-bit terms, x ~ x0 + x1 (+ x2),
// x0 = rn(x), x1 = rn(x - x0), x2 = rn(x - x0 - x1), and a real product is
// the sum of the term products that matter at float32 accuracy:
//   NT = 2:  a0 b0 + a0 b1 + a1 b0                      (3 MFMAs)
//   NT = 3:  a0 b0 + a0 b1 + a1 b0 + a0 b2 + a1 b1 + a2 b0   (6 MFMAs)
// accumulated in float32.  Complex products use four real products
// (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br); -Ai is formed in registers by
// flipping sign bits.
//
// Layout: both operands as 16-bit planes [re/im][term] of a [row][K]
// matrix, stored k-blocked (blocks of kKB = 32 k for all rows, so a stage of
// a row tile is one contiguous run of whole cache lines):
//   forward   A = Omega_r [Urp][Rp],      B^T = P^T [Cp][Rp]
//   adjoint   A = Omega_r^H [Rp][Urp],    B^T = S^T [Cp][Urp]
// and each MFMA operand fragment (8 consecutive k of one row) is one 16-byte
// LDS read.  A stage holds BK complex k (BK / 16 MFMA k-steps) in rows of
// BK / 8 16-byte chunks; the chunk index is XOR-swizzled with row bits so
// fragment reads of 8 or 16 consecutive rows hit distinct banks.
//
// Scheduling, split-K tail and in-order reduction as in the float32 kernel.
// Epilogues: store float32 C (forward, for the focus gather); or project onto
// the amplitude constraint and write the pupil field directly as the split
// B^T planes of the next forward product, transposed through LDS so every
// store is a 16-byte run of one row of P^T.
#include <cstring>

#include "gswmtp_internal.h"

namespace gswmtp {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int kKStep = 16;     // k per MFMA instruction

template <bool BF>
__device__ __forceinline__ v16f mfma16(u4 a, u4 b, v16f c) {
  if constexpr (BF)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a),
                                                  __builtin_bit_cast(v8h, b), c, 0, 0, 0);
}

// Chunk swizzle of an LDS row of CH 16-byte chunks (a permutation of the
// chunks of each row; conflict-free fragment reads for 32 and 64 banks).
template <int CH>
__device__ __forceinline__ int swz(int row) {
  if constexpr (CH == 2) return ((row >> 2) ^ (row >> 3)) & 1;
  return ((row >> 1) & 1) ^ (((row >> 2) & 1) << 1) ^ ((row >> 3) & 1);
}

template <int BM, int BN, int BK, int NT, int EPI, int PIPE = 0>
constexpr int split_lds_bytes() {
  // two stages of every operand plane held in LDS (the direct loop: A only)
  constexpr int ops = 2 * 2 * NT * (BM + (PIPE == 2 ? 0 : BN)) * (BK / 8) * 16;
  constexpr int tr = EPI == EPI_PROJECT   ? 2 * NT * BN * (BM + 8) * 2
                     : EPI == EPI_GATHER ? gather_lds_bytes<BM, BN>()
                                         : 0;
  return ops > tr ? ops : tr;
}

__device__ __forceinline__ int xcd_tile(int bid, int tiles) {
  const int xcd = bid & 7, local = bid >> 3;
  const int per = tiles >> 3, rem = tiles & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

struct SplitArgs {
  const unsigned short *__restrict__ a;   // [2][NT][M][K]
  const unsigned short *__restrict__ b;   // [2][NT][N][K]
  size_t a_plane, b_plane;                // elements per plane
  int M, N, K;
  float *cr;                              // EPI_STORE: float32 planes [M][ldc]
  float *ci;
  int ldc;
  const float *__restrict__ amp;          // EPI_PROJECT: amplitude [M][ldc]
  unsigned short *pt;                     // EPI_PROJECT: split planes [2][NT][N][M]
  size_t pt_plane;
  const int *done;
  float *part;
  GatherCtx g;                            // EPI_GATHER
  int phase;                              // 0: tiles and K chunks; 1: reduce tail chunks
  int tiles_m, t_dp, split;
  int xgm;                                // 16x16-block loop: XCD groups along M (<= 1: none)
};

// Operand fragments of one MFMA k-step for the wave's MB x NB blocks: lane
// (l32, h) holds row l32 of its block, k = 16 ks + 8 h .. + 7, every plane.
template <int BM, int BN, int NT>
struct Frags {
  u4 a[BM / 64][2 * NT];
  u4 b[BN / 64][2 * NT];
};

template <int BM, int BN, int BK, int NT>
__device__ __forceinline__ void load_frags(const u4 *qa, const u4 *qb, int ks, int wm, int wn,
                                           int l32, int h, Frags<BM, BN, NT> &f) {
  constexpr int WTM = BM / 2, WTN = BN / 2, MB = WTM / 32, NB = WTN / 32;
  constexpr int PL = 2 * NT, CH = BK / 8;
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int row = wm * WTM + i * 32 + l32;
#pragma unroll
    for (int pl = 0; pl < PL; ++pl)
      f.a[i][pl] = qa[(pl * BM + row) * CH + ((2 * ks + h) ^ swz<CH>(row))];
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int row = wn * WTN + j * 32 + l32;
#pragma unroll
    for (int pl = 0; pl < PL; ++pl)
      f.b[j][pl] = qb[(pl * BN + row) * CH + ((2 * ks + h) ^ swz<CH>(row))];
  }
}

// The MFMAs of one k-step: term pairs (ta, tb) with ta + tb < NT, small
// terms first; -Ai Bi by flipping the sign bits of the imaginary terms of A (NEGB: of B,
// for B fragments that sit in registers long before their MFMAs, so the
// flips never wait on a fresh LDS read); the same products either way.
template <int MB, int NB, bool BF, int NT, bool NEGB = false>
__device__ __forceinline__ void mma_ab(const u4 (&fa)[MB][2 * NT], const u4 (&fb)[NB][2 * NT],
                                       v16f (&accR)[MB][NB], v16f (&accI)[MB][NB]) {
  constexpr int NX = NEGB ? NB : MB;
  u4 nx[NX][NT];
#pragma unroll
  for (int i = 0; i < NX; ++i)
#pragma unroll
    for (int q = 0; q < NT; ++q) nx[i][q] = (NEGB ? fb[i][NT + q] : fa[i][NT + q]) ^ 0x80008000u;
  // Each accumulator takes its products in the same order (per term pair:
  // real part Ar Br then -Ai Bi, imaginary part Ar Bi then Ai Br); the
  // accumulators are interleaved so that consecutive MFMAs are independent.
#pragma unroll
  for (int s = NT - 1; s >= 0; --s)
#pragma unroll
    for (int ta = 0; ta <= s; ++ta) {
      const int tb = s - ta;
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          accR[i][j] = mfma16<BF>(fa[i][ta], fb[j][tb], accR[i][j]);
          accI[i][j] = mfma16<BF>(fa[i][ta], fb[j][NT + tb], accI[i][j]);
        }
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          if constexpr (NEGB)
            accR[i][j] = mfma16<BF>(fa[i][NT + ta], nx[j][tb], accR[i][j]);
          else
            accR[i][j] = mfma16<BF>(nx[i][ta], fb[j][NT + tb], accR[i][j]);
          accI[i][j] = mfma16<BF>(fa[i][NT + ta], fb[j][tb], accI[i][j]);
        }
    }
}

template <int BM, int BN, bool BF, int NT>
__device__ __forceinline__ void mma_frags(const Frags<BM, BN, NT> &f,
                                          v16f (&accR)[BM / 64][BN / 64],
                                          v16f (&accI)[BM / 64][BN / 64]) {
  mma_ab<BM / 64, BN / 64, BF, NT>(f.a, f.b, accR, accI);
}

// Scheduling requests for the pipelined loop (instruction classes of
// sched_group_barrier: 0x008 MFMA, 0x020 VMEM read, 0x100 DS read, 0x200 DS
// write).  N pairs of (one DS read, one MFMA).
template <int N>
__device__ __forceinline__ void sched_read_mfma() {
  if constexpr (N > 0) {
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    sched_read_mfma<N - 1>();
  }
}
// N groups of (W DS writes, one MFMA).
template <int N, int W>
__device__ __forceinline__ void sched_write_mfma() {
  if constexpr (N > 0) {
    __builtin_amdgcn_sched_group_barrier(0x200, W, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    sched_write_mfma<N - 1, W>();
  }
}

// N pairs of (one VMEM read, one MFMA).
template <int N>
__device__ __forceinline__ void sched_vmem_mfma() {
  if constexpr (N > 0) {
    __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    sched_vmem_mfma<N - 1>();
  }
}

// MFMA work of one LDS stage: BK / 16 k-steps over the wave's MB x NB blocks.
// With KG k-groups the stage's k-steps are dealt out in KG contiguous runs:
// group kg takes k-steps kg KS / KG .. (kg + 1) KS / KG - 1.
template <int BM, int BN, int BK, bool BF, int NT, int KG>
__device__ __forceinline__ void stage_mma(const u4 *qa, const u4 *qb,
                                          v16f (&accR)[BM / 64][BN / 64],
                                          v16f (&accI)[BM / 64][BN / 64], int wm, int wn,
                                          int l32, int h, int kg) {
  constexpr int KS = BK / kKStep, KSG = KS / KG;
  static_assert(KS % KG == 0, "k-steps per stage must divide among the k-groups");
#pragma unroll
  for (int q_ = 0; q_ < KSG; ++q_) {
    Frags<BM, BN, NT> f;
    load_frags<BM, BN, BK, NT>(qa, qb, kg * KSG + q_, wm, wn, l32, h, f);
    mma_frags<BM, BN, BF, NT>(f, accR, accI);
  }
}

// KG = 2: two k-groups of four waves each (512 threads) share every LDS
// stage, each multiplying half of its k-steps into its own accumulators;
// after the last stage group 1 hands its sums to group 0 through LDS
// (group 0 adds them: acc0 + acc1, a fixed order) and exits, and group 0
// runs the epilogue alone (a barrier waits only for the waves still
// running).  The tile count of these products is small (about two 64 x 64
// tiles per CU), so this doubles the waves per SIMD that hide LDS and
// barrier latency without shrinking the tiles.
//
// PIPE (one k-group, two k-steps per stage): the fragment reads are
// software-pipelined so LDS traffic overlaps the MFMAs of the same wave.
// Per stage S (LDS buffer S & 1, fragments of k-step 0 already in f0): read
// k-step 1 into f1 while f0's MFMAs run; one barrier (every read of the
// buffer is done, stage S + 1 is published); read stage S + 1's k-step 0
// into f0 while f1's MFMAs run; then store stage S + 2 (held in registers
// since two stages ago) into the buffer just left and issue the loads of
// stage S + 4.
template <int BM, int BN, int BK, bool BF, int NT, int EPI, int KG, int PIPE>
constexpr int split_lds_u4() {
  return (split_lds_bytes<BM, BN, BK, NT, EPI, PIPE>() + 15) / 16;
}

// The direct loop (two terms, 64 x 128 tiles): the four waves side by side
// along N, each owning BN/4 rows of B^T, which it loads straight from HBM
// into its MFMA fragment registers four stages ahead (no two waves read the
// same B row, so B needs no LDS); A is shared through two LDS stages as in
// the pipelined loop (a deeper A prefetch, four stages, measured no
// faster).  Per stage S (LDS buffer S & 1, B register set S % 4, A
// fragments of k-step 0 already in f0): read A's k-step 1 into f1 while
// f0's MFMAs run; one barrier; read stage S + 1's k-step 0 into f0 while
// f1's MFMAs run; store stage S + 2 of A (in registers since two stages ago)
// into the buffer just left and issue the loads of stage S + 4 of A and B.
// Returns false when the done flag stops the product.
template <int BM, int BK, int NT>
__device__ __forceinline__ void load_fa(const u4 *qa, int ks, int l32, int h,
                                        u4 (&fa)[BM / 32][2 * NT]) {
  constexpr int CH = BK / 8;
#pragma unroll
  for (int i = 0; i < BM / 32; ++i) {
    const int row = i * 32 + l32;
#pragma unroll
    for (int pl = 0; pl < 2 * NT; ++pl)
      fa[i][pl] = qa[(pl * BM + row) * CH + ((2 * ks + h) ^ swz<CH>(row))];
  }
}

template <int BM, int BN, int BK, bool BF, int NT, bool PRE>
__device__ __forceinline__ bool direct_loop(const SplitArgs &a, int m0, int n0, int kb, int ke,
                                            int tid, u4 *lds, v16f (&accR)[BM / 32][1],
                                            v16f (&accI)[BM / 32][1], GatherPre &gp) {
  using L = WaveLayout<BM, BN, true>;
  constexpr int MB = L::MB, PL = 2 * NT, KS = BK / kKStep, CH = BK / 8;
  static_assert(L::NB == 1 && KS == 2 && BK == kKB, "direct loop: 32 B rows per wave, one k-block per stage");
  constexpr int LA = PL * BM * CH, NA = LA / kThreads;
  static_assert(LA % kThreads == 0, "tile/thread mismatch");
  constexpr int SA_SZ = LA;
  u4 *sA = lds;
  const int lane = tid & 63, wave = tid >> 6, l32 = lane & 31, h = lane >> 5;
  const unsigned short *ga[NA];
  int la[NA];
#pragma unroll
  for (int s = 0; s < NA; ++s) {
    const int id = tid + kThreads * s;
    const int c = id % CH, row = (id / CH) % BM, plane = id / (CH * BM);
    ga[s] = a.a + (size_t)plane * a.a_plane + (size_t)(m0 + row) * kKB + 8 * c;
    la[s] = (plane * BM + row) * CH + (c ^ swz<CH>(row));
  }
  // B^T row of lane (l32, h): n0 + WTN wave + l32; it holds k 8h .. 8h + 7 of each k-step
  const unsigned short *gb = a.b + (size_t)(n0 + L::WTN * wave + l32) * kKB + 8 * h;
  if (kb >= ke) return !(a.done && *a.done);
  const int last = ke - 1;
  u4 ra0[NA], ra1[NA];
  u4 bq0[KS][1][PL], bq1[KS][1][PL], bq2[KS][1][PL], bq3[KS][1][PL];
#define D_LOAD_A(RA, KT)                                                                   \
  do {                                                                                     \
    const size_t k_ = (size_t)(KT) * BK;                                                   \
    const size_t o_ = k_ / kKB * ((size_t)a.M * kKB) + k_ % kKB;                           \
    _Pragma("unroll") for (int s_ = 0; s_ < NA; ++s_) RA[s_] =                             \
        *reinterpret_cast<const u4 *>(ga[s_] + o_);                                        \
  } while (0)
#define D_LOAD_B(BQ, KT)                                                                   \
  do {                                                                                     \
    _Pragma("unroll") for (int ks_ = 0; ks_ < KS; ++ks_) {                                 \
      const size_t k_ = (size_t)(KT) * BK + ks_ * kKStep;                                  \
      const size_t o_ = k_ / kKB * ((size_t)a.N * kKB) + k_ % kKB;                         \
      _Pragma("unroll") for (int pl_ = 0; pl_ < PL; ++pl_) BQ[ks_][0][pl_] =               \
          *reinterpret_cast<const u4 *>(gb + pl_ * a.b_plane + o_);                        \
    }                                                                                      \
  } while (0)
#define D_STORE_A(RA, BUF)                                                                 \
  do {                                                                                     \
    _Pragma("unroll") for (int s_ = 0; s_ < NA; ++s_) sA[(BUF) * SA_SZ + la[s_]] = RA[s_]; \
  } while (0)
  D_LOAD_A(ra0, kb);
  D_LOAD_A(ra1, kb + 1 < last ? kb + 1 : last);
  D_LOAD_B(bq0, kb);
  D_LOAD_B(bq1, kb + 1 < last ? kb + 1 : last);
  D_LOAD_B(bq2, kb + 2 < last ? kb + 2 : last);
  D_LOAD_B(bq3, kb + 3 < last ? kb + 3 : last);
  if constexpr (PRE) gather_pre_foci(a.g, m0, tid, gp);   // behind the operand loads
  const int stop = a.done ? *a.done : 0;
  asm volatile("" ::: "memory");
  if (stop) return false;
  D_STORE_A(ra0, 0);
  D_LOAD_A(ra0, kb + 2 < last ? kb + 2 : last);
  D_STORE_A(ra1, 1);
  D_LOAD_A(ra1, kb + 3 < last ? kb + 3 : last);
  __syncthreads();
  u4 f0[MB][PL], f1[MB][PL];
  load_fa<BM, BK, NT>(sA, 0, l32, h, f0);
  // per k-step: NR fragment reads, NM MFMAs; per stage NA stores and NV loads
  constexpr int NR = MB * PL, NM = MB * 2 * NT * (NT + 1), NV = NA + KS * PL;
  static_assert(NM >= NR + NA, "interleave pattern");
  constexpr int NVM = NV < NM - NR - NA ? NV : NM - NR - NA;   // (load, MFMA) pairs
#define D_STEP(BUF, RA, BQ, S)                                                            \
  do {                                                                                    \
    load_fa<BM, BK, NT>(sA + (BUF) * SA_SZ, 1, l32, h, f1);                               \
    mma_ab<MB, 1, BF, NT, true>(f0, BQ[0], accR, accI);                                   \
    sched_read_mfma<NR>();                                                                \
    __builtin_amdgcn_sched_group_barrier(0x008, NM - NR, 0);                              \
    __syncthreads();                                                                      \
    __builtin_amdgcn_sched_barrier(0);                                                    \
    load_fa<BM, BK, NT>(sA + (1 - (BUF)) * SA_SZ, 0, l32, h, f0);                         \
    mma_ab<MB, 1, BF, NT, true>(f1, BQ[1], accR, accI);                                   \
    D_STORE_A(RA, BUF);                                                                   \
    D_LOAD_A(RA, (S) + 4 < last ? (S) + 4 : last);                                        \
    D_LOAD_B(BQ, (S) + 4 < last ? (S) + 4 : last);                                        \
    sched_read_mfma<NR>();                                                                \
    sched_write_mfma<NA, 1>();                                                            \
    sched_vmem_mfma<NVM>();                                                               \
    if constexpr (NM - NR - NA - NVM > 0)                                                 \
      __builtin_amdgcn_sched_group_barrier(0x008, NM - NR - NA - NVM, 0);                 \
    if constexpr (NV - NVM > 0) __builtin_amdgcn_sched_group_barrier(0x020, NV - NVM, 0); \
    __builtin_amdgcn_sched_barrier(0);                                                    \
  } while (0)
  int kt = kb;
  for (; kt + 3 < ke; kt += 4) {
    D_STEP(0, ra0, bq0, kt);
    D_STEP(1, ra1, bq1, kt + 1);
    D_STEP(0, ra0, bq2, kt + 2);
    D_STEP(1, ra1, bq3, kt + 3);
  }
  if (kt < ke) D_STEP(0, ra0, bq0, kt);
  if (kt + 1 < ke) D_STEP(1, ra1, bq1, kt + 1);
  if (kt + 2 < ke) D_STEP(0, ra0, bq2, kt + 2);
#undef D_STEP
#undef D_LOAD_A
#undef D_LOAD_B
#undef D_STORE_A
  return true;
}

// One unit of a product: tile t over K stages [kb, ke) (LDS `lds` of
// split_lds_u4 entries).  tail < 0: the epilogue runs on the sums (a forward
// tile's gather writes partial row prow, -1: n0 / BN); tail >= 0 in phase 0:
// chunk `chunk` of tail tile `tail` stores its partial tile; phase 1 (kb =
// ke): tail tile `tail` adds its chunks' partials in order and runs the
// epilogue.
template <int BM, int BN, int BK, bool BF, int NT, int EPI, int KG, int PIPE>
__device__ __forceinline__ void cgemm_split_unit(const SplitArgs &a, const int t, const int kb,
                                                 const int ke, const int tail, const int chunk,
                                                 const int prow, u4 *lds) {
  constexpr int NTH = kThreads * KG;
  using L = WaveLayout<BM, BN, PIPE == 2>;
  constexpr int WTM = L::WTM, WTN = L::WTN;
  constexpr int MB = L::MB, NB = L::NB;
  constexpr int PL = 2 * NT;                     // planes per operand
  constexpr int CH = BK / 8;                     // 16-byte chunks per row and stage
  constexpr int LA = PL * BM * CH, LB = PL * BN * CH;   // chunks loaded per stage
  constexpr int NA = LA / NTH, NBL = LB / NTH;
  static_assert(LA % NTH == 0 && LB % NTH == 0, "tile/thread mismatch");
  constexpr int SA_SZ = LA, SB_SZ = LB;
  // epilogue transpose tile: [plane][n][m] 16-bit with rows padded by 8 elements
  constexpr int TP = BM + 8;

  u4 *sA = lds;                         // [2][SA_SZ]
  u4 *sB = lds + 2 * SA_SZ;             // [2][SB_SZ]

  const int tid = threadIdx.x;
  const int m0 = (t % a.tiles_m) * BM;
  const int n0 = (t / a.tiles_m) * BN;
  const int lane = tid & 63, wave = (tid >> 6) & 3, kg = tid >> 8;
  const int wm = L::wm(wave), wn = L::wn(wave);
  const int l32 = lane & 31, h = lane >> 5;

  v16f accR[MB][NB], accI[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      accR[i][j] = v16f{0};
      accI[i][j] = v16f{0};
    }

  // the gather's focus indices: row range now, foci behind the operand loads
  GatherPre gp;
  if constexpr (EPI == EPI_GATHER) gather_pre_rows(a.g, m0, BM, gp);
  // the projection's amplitudes, read now and used after the main loop
  // (whole tiles only: K-chunk blocks write partials)
  float ampv[EPI == EPI_PROJECT ? MB : 1][EPI == EPI_PROJECT ? NB : 1][16];
  if constexpr (EPI == EPI_PROJECT) {
    if (tail < 0) {
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int ml = wm * WTM + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
            ampv[i][j][r] = a.amp[(size_t)(m0 + ml) * a.ldc + n0 + wn * WTN + j * 32 + l32];
          }
    }
  }
  if constexpr (PIPE == 2) {
    static_assert(KG == 1, "direct loop: one k-group");
    if (!direct_loop<BM, BN, BK, BF, NT, EPI == EPI_GATHER>(a, m0, n0, kb, ke, tid, lds, accR,
                                                             accI, gp))
      return;
    __syncthreads();   // the epilogues reuse the operand buffers
  } else {
  // staging: chunk id = (plane * rows + row) * CH + c (16 bytes, 8 k values)
  const unsigned short *ga[NA];
  const unsigned short *gb[NBL];
  int la[NA], lb[NBL];
#pragma unroll
  for (int s = 0; s < NA; ++s) {
    const int id = tid + NTH * s;
    const int c = id % CH, row = (id / CH) % BM, plane = id / (CH * BM);
    ga[s] = a.a + (size_t)plane * a.a_plane + (size_t)(m0 + row) * kKB + 8 * c;
    la[s] = (plane * BM + row) * CH + (c ^ swz<CH>(row));
  }
#pragma unroll
  for (int s = 0; s < NBL; ++s) {
    const int id = tid + NTH * s;
    const int c = id % CH, row = (id / CH) % BN, plane = id / (CH * BN);
    gb[s] = a.b + (size_t)plane * a.b_plane + (size_t)(n0 + row) * kKB + 8 * c;
    lb[s] = (plane * BN + row) * CH + (c ^ swz<CH>(row));
  }
  // Two stages in flight: while stage kt is multiplied out of LDS buffer
  // (kt - kb) & 1, the register set of stage kt + 1 waits to be written to
  // the other buffer and the loads of stage kt + 2 are issued into the set
  // just freed.  Loads and stores are unconditional (stage indices clamped
  // to the last stage; the extra copies land in a buffer nobody reads), so
  // every store waits only for its own set's loads, never for the set issued
  // after it.
  u4 r0a[NA], r0b[NBL], r1a[NA], r1b[NBL];
  // stage kt starts at k = kt BK: k-block (kt BK) / kKB, offset (kt BK) % kKB
#define LOAD_STAGE(RA, RB, KT)                                                         \
  do {                                                                                 \
    const size_t k_ = (size_t)(KT) * BK;                                               \
    const size_t oa_ = k_ / kKB * ((size_t)a.M * kKB) + k_ % kKB;                      \
    const size_t ob_ = k_ / kKB * ((size_t)a.N * kKB) + k_ % kKB;                      \
    _Pragma("unroll") for (int s_ = 0; s_ < NA; ++s_) RA[s_] =                         \
        *reinterpret_cast<const u4 *>(ga[s_] + oa_);                                   \
    _Pragma("unroll") for (int s_ = 0; s_ < NBL; ++s_) RB[s_] =                        \
        *reinterpret_cast<const u4 *>(gb[s_] + ob_);                                   \
  } while (0)
#define STORE_STAGE(RA, RB, BUF)                                                       \
  do {                                                                                 \
    _Pragma("unroll") for (int s_ = 0; s_ < NA; ++s_) sA[(BUF) * SA_SZ + la[s_]] = RA[s_]; \
    _Pragma("unroll") for (int s_ = 0; s_ < NBL; ++s_) sB[(BUF) * SB_SZ + lb[s_]] = RB[s_]; \
  } while (0)
  if (kb < ke) {
    const int last = ke - 1;
    LOAD_STAGE(r0a, r0b, kb);
    LOAD_STAGE(r1a, r1b, kb + 1 < last ? kb + 1 : last);
    if constexpr (EPI == EPI_GATHER) gather_pre_foci(a.g, m0, tid, gp);
    // The done flag is read while the first two stages are in flight (the
    // loads are kept above the test), not before them.
    const int stop = a.done ? *a.done : 0;
    asm volatile("" ::: "memory");
    if (stop) return;
    if constexpr (PIPE == 1) {
      static_assert(KG == 1 && BK == 2 * kKStep, "pipelined loop: one group, two k-steps");
      STORE_STAGE(r0a, r0b, 0);
      LOAD_STAGE(r0a, r0b, kb + 2 < last ? kb + 2 : last);
      STORE_STAGE(r1a, r1b, 1);
      LOAD_STAGE(r1a, r1b, kb + 3 < last ? kb + 3 : last);
      __syncthreads();
      Frags<BM, BN, NT> f0, f1;
      load_frags<BM, BN, BK, NT>(sA, sB, 0, wm, wn, l32, h, f0);
      // per k-step: NR fragment reads, NM MFMAs; NS stage stores / loads per thread
      constexpr int NR = (BM / 64 + BN / 64) * 2 * NT;
      constexpr int NM = (BM / 64) * (BN / 64) * 2 * NT * (NT + 1);
      constexpr int NS = NA + NBL;
      static_assert(NM >= NR, "interleave pattern");
      constexpr int NW = NS < NM - NR ? NS : NM - NR;   // (store, MFMA) pairs
      // The read of the next stage's k-step 0 is unconditional: after the
      // last stage it reads the clamped copy in the other buffer, unused.
#define PIPE_STEP(BUF, RA, RB, S)                                                              \
  do {                                                                                         \
    load_frags<BM, BN, BK, NT>(sA + (BUF) * SA_SZ, sB + (BUF) * SB_SZ, 1, wm, wn, l32, h, f1); \
    mma_frags<BM, BN, BF, NT>(f0, accR, accI);                                                 \
    sched_read_mfma<NR>();                                                                     \
    __builtin_amdgcn_sched_group_barrier(0x008, NM - NR, 0);                                   \
    __syncthreads();                                                                           \
    __builtin_amdgcn_sched_barrier(0);                                                         \
    load_frags<BM, BN, BK, NT>(sA + (1 - (BUF)) * SA_SZ, sB + (1 - (BUF)) * SB_SZ, 0, wm, wn,   \
                               l32, h, f0);                                                    \
    mma_frags<BM, BN, BF, NT>(f1, accR, accI);                                                 \
    STORE_STAGE(RA, RB, BUF);                                                                  \
    LOAD_STAGE(RA, RB, (S) + 4 < last ? (S) + 4 : last);                                       \
    sched_read_mfma<NR>();                                                                     \
    sched_write_mfma<NW, 1>();                                                                 \
    if constexpr (NM - NR - NW > 0) __builtin_amdgcn_sched_group_barrier(0x008, NM - NR - NW, 0); \
    if constexpr (NS - NW > 0) __builtin_amdgcn_sched_group_barrier(0x200, NS - NW, 0);       \
    __builtin_amdgcn_sched_group_barrier(0x020, NS, 0);                                        \
    __builtin_amdgcn_sched_barrier(0);                                                         \
  } while (0)
      int kt = kb;
      for (; kt + 1 < ke; kt += 2) {
        PIPE_STEP(0, r0a, r0b, kt);
        PIPE_STEP(1, r1a, r1b, kt + 1);
      }
      if (kt < ke) PIPE_STEP(0, r0a, r0b, kt);
#undef PIPE_STEP
    } else {
      // Stages in pairs with one exit, so the loop is entered from the
      // prologue and from its back edge in the same state (set 0 older, set 1
      // newer, both in flight); an odd last stage follows the loop.
      int kt = kb;
      for (; kt + 1 < ke; kt += 2) {
        STORE_STAGE(r0a, r0b, 0);
        __syncthreads();
        LOAD_STAGE(r0a, r0b, kt + 2 < last ? kt + 2 : last);
        __builtin_amdgcn_sched_barrier(0);   // issue the loads here, ahead of the MFMAs
        stage_mma<BM, BN, BK, BF, NT, KG>(sA, sB, accR, accI, wm, wn, l32, h, kg);
        STORE_STAGE(r1a, r1b, 1);
        __syncthreads();
        LOAD_STAGE(r1a, r1b, kt + 3 < last ? kt + 3 : last);
        __builtin_amdgcn_sched_barrier(0);
        stage_mma<BM, BN, BK, BF, NT, KG>(sA + SA_SZ, sB + SB_SZ, accR, accI, wm, wn, l32, h,
                                          kg);
      }
      if (kt < ke) {
        STORE_STAGE(r0a, r0b, 0);
        __syncthreads();
        stage_mma<BM, BN, BK, BF, NT, KG>(sA, sB, accR, accI, wm, wn, l32, h, kg);
      }
    }
    __syncthreads();   // the epilogues reuse the operand buffers
    if constexpr (KG == 2) {
      // group 1's sums to group 0, thread-major (one float per lane per store)
      float *red = reinterpret_cast<float *>(lds);
      const int t4 = tid & (kThreads - 1);
      if (kg == 1) {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int o = (((i * NB + j) * 16 + r) * 2) * kThreads + t4;
              red[o] = accR[i][j][r];
              red[o + kThreads] = accI[i][j][r];
            }
      }
      __syncthreads();
      if (kg == 1) return;
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int o = (((i * NB + j) * 16 + r) * 2) * kThreads + t4;
            accR[i][j][r] += red[o];
            accI[i][j][r] += red[o + kThreads];
          }
      __syncthreads();   // the reduction buffer is read before any epilogue writes
    }
  } else {
    const int stop = a.done ? *a.done : 0;
    if (stop) return;
  }
  if constexpr (KG == 2)
    if (kg == 1) return;   // tail-reduction blocks: group 0 alone
#undef LOAD_STAGE
#undef STORE_STAGE
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

  // epilogue; accumulator item r of lane (l32, h): row 8 (r/4) + 4 h + r % 4, column l32
  if constexpr (EPI == EPI_GATHER) {
    gather_epilogue<BM, BN, PIPE == 2>(a.g, accR, accI, reinterpret_cast<float *>(lds), m0, n0,
                                       tid, gp, prow);
  } else if constexpr (EPI == EPI_STORE) {
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int n = n0 + wn * WTN + j * 32 + l32;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const size_t o = (size_t)(m0 + wm * WTM + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3)) *
                               a.ldc + n;
          a.cr[o] = accR[i][j][r];
          a.ci[o] = accI[i][j][r];
        }
      }
  } else if constexpr (EPI == EPI_PROJECT) {
    // project, split into terms, transpose the tile through LDS, then write
    // rows of P^T [plane][n][m0 .. m0 + BM) in 16-byte runs
    unsigned short *tt = reinterpret_cast<unsigned short *>(lds);
    __syncthreads();   // operand stages are no longer read
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int nl = wn * WTN + j * 32 + l32;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int ml = wm * WTM + i * 32 + 8 * g + 4 * h;
          unsigned short tr[NT][4], ti[NT][4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float cr = accR[i][j][4 * g + q], ci = accI[i][j][4 * g + q];
            float pr, pi;
            const float am = tail < 0 ? ampv[i][j][4 * g + q]
                                      : a.amp[(size_t)(m0 + ml + q) * a.ldc + n0 + nl];
            project_amp(cr, ci, am, pr, pi);
            split_terms<BF, NT>(pr, &tr[0][q], 4);
            split_terms<BF, NT>(pi, &ti[0][q], 4);
          }
#pragma unroll
          for (int s = 0; s < NT; ++s) {
            const u2 vr = {(unsigned)tr[s][0] | ((unsigned)tr[s][1] << 16),
                           (unsigned)tr[s][2] | ((unsigned)tr[s][3] << 16)};
            const u2 vi = {(unsigned)ti[s][0] | ((unsigned)ti[s][1] << 16),
                           (unsigned)ti[s][2] | ((unsigned)ti[s][3] << 16)};
            *reinterpret_cast<u2 *>(tt + ((size_t)s * BN + nl) * TP + ml) = vr;
            *reinterpret_cast<u2 *>(tt + ((size_t)(NT + s) * BN + nl) * TP + ml) = vi;
          }
        }
      }
    __syncthreads();
    constexpr int RC = BM / 8;                  // 16-byte chunks per row
    constexpr int NCH = PL * BN * RC;
    static_assert(NCH % kThreads == 0, "epilogue chunking");
#pragma unroll
    for (int s = 0; s < NCH / kThreads; ++s) {
      const int id = tid + kThreads * s;
      const int c = id % RC, nl = (id / RC) % BN, pl = id / (RC * BN);
      const u4 v = *reinterpret_cast<const u4 *>(tt + ((size_t)pl * BN + nl) * TP + 8 * c);
      *reinterpret_cast<u4 *>(a.pt + (size_t)pl * a.pt_plane +
                              kblk_index(n0 + nl, m0 + 8 * c, a.N)) = v;   // 8 m, one k-block
    }
  }
}

// The product for block `bid` of one schedule (whole tile, K chunk or tail
// reduction).
template <int BM, int BN, int BK, bool BF, int NT, int EPI, int KG, int PIPE>
__device__ __forceinline__ void cgemm_split_body(const SplitArgs &a, const int bid, u4 *lds) {
  const int KT = a.K / BK;
  if (a.phase == 1) {
    cgemm_split_unit<BM, BN, BK, BF, NT, EPI, KG, PIPE>(a, a.t_dp + bid, 0, 0, bid, 0, -1, lds);
  } else if (bid < a.t_dp) {
    cgemm_split_unit<BM, BN, BK, BF, NT, EPI, KG, PIPE>(a, xcd_tile(bid, a.t_dp), 0, KT, -1, 0,
                                                        -1, lds);
  } else {
    const int u = bid - a.t_dp, tail = u / a.split, chunk = u % a.split;
    cgemm_split_unit<BM, BN, BK, BF, NT, EPI, KG, PIPE>(a, a.t_dp + tail, chunk * KT / a.split,
                                                        (chunk + 1) * KT / a.split, tail, chunk,
                                                        -1, lds);
  }
}

template <int BM, int BN, int BK, bool BF, int NT, int EPI, int KG, int PIPE>
__global__ __launch_bounds__(kThreads * KG) void cgemm_split_mfma(SplitArgs a) {
  __shared__ u4 lds[split_lds_u4<BM, BN, BK, BF, NT, EPI, KG, PIPE>()];
  cgemm_split_body<BM, BN, BK, BF, NT, EPI, KG, PIPE>(a, blockIdx.x, lds);
}

// Work-list launch (batched form): workgroup b runs the units off[b] ..
// off[b + 1] - 1 of the list (a persistent grid, the ranges balanced on the
// host), or unit b alone when off is null; each unit is a tile (or the K
// chunk of a forward tile) of one plan's product; the LDS is reused from unit
// to unit behind a barrier.
template <int BM, int BN, int BK, bool BF, int NT, int EPI, int KG, int PIPE>
__global__ __launch_bounds__(kThreads * KG) void cgemm_split_work(const SplitArgs *items,
                                                                  const WorkUnit *work, const int *off, int n) {
  __shared__ u4 lds[split_lds_u4<BM, BN, BK, BF, NT, EPI, KG, PIPE>()];
  // units off[b] .. off[b + 1] - 1 (persistent), or unit b (off null)
  const int w0 = off ? off[blockIdx.x] : (int)blockIdx.x;
  const int w1 = off ? off[blockIdx.x + 1] : w0 + 1;
  for (int w = w0; w < w1 && w < n; ++w) {
    if (w != w0) __syncthreads();   // the previous unit's LDS reads are done
    const WorkUnit u = work[w];
    cgemm_split_unit<BM, BN, BK, BF, NT, EPI, KG, PIPE>(items[u.item], u.tile, u.kb, u.ke, -1, 0,
                                                        u.prow, lds);
  }
}

// Split-K tail with the projection epilogue: adds the K-chunk partials of
// each tail tile in chunk order and projects, then writes the 16-bit term
// planes of P^T (four consecutive rows of one column per thread: one 8-byte
// store per plane).  Block (tail, g) covers slots r = 4g .. 4g + 3 of every
// (i, j) block of the tile.
template <int BM, int BN, bool BF, int NT, bool COLS>
__global__ __launch_bounds__(kThreads) void cgemm_tail_project_split(SplitArgs a) {
  constexpr int MB = WaveLayout<BM, BN, COLS>::MB, NB = WaveLayout<BM, BN, COLS>::NB;
  constexpr int unit = 2 * MB * NB * 16 * kThreads;
  const int tail = blockIdx.x, g = blockIdx.y, tid = threadIdx.x;
  const int t = a.t_dp + tail;
  const int m0 = (t % a.tiles_m) * BM, n0 = (t / a.tiles_m) * BN;
  const float *pt = a.part + (size_t)tail * a.split * unit + tid;
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      int m, n;
      tile_slot_pos<BM, BN, COLS>(tid, i, j, 4 * g, m, n);   // rows m .. m + 3, column n
      float av[4];   // amplitudes read with the partials, not after them
#pragma unroll
      for (int q = 0; q < 4; ++q) av[q] = a.amp[(size_t)(m0 + m + q) * a.ldc + n0 + n];
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
      unsigned short tr[NT][4], ti[NT][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float pr, pi;
        project_amp(sr[q], si[q], av[q], pr, pi);
        split_terms<BF, NT>(pr, &tr[0][q], 4);
        split_terms<BF, NT>(pi, &ti[0][q], 4);
      }
      const size_t base = kblk_index(n0 + n, m0 + m, a.N);   // rows m .. m + 3, one k-block
#pragma unroll
      for (int s = 0; s < NT; ++s) {
        const u2 vr = {(unsigned)tr[s][0] | ((unsigned)tr[s][1] << 16),
                       (unsigned)tr[s][2] | ((unsigned)tr[s][3] << 16)};
        const u2 vi = {(unsigned)ti[s][0] | ((unsigned)ti[s][1] << 16),
                       (unsigned)ti[s][2] | ((unsigned)ti[s][3] << 16)};
        *reinterpret_cast<u2 *>(a.pt + (size_t)s * a.pt_plane + base) = vr;
        *reinterpret_cast<u2 *>(a.pt + (size_t)(NT + s) * a.pt_plane + base) = vi;
      }
    }
}

// ---------------------------------------------------------------------------
// The 16x16-block loop: tiles of BM x BN with BM a multiple of 16 (e.g.
// 48 x 192, which covers a 1152 x 1920 product in 240 tiles, one round on
// 256 CUs, where 64 x 64 tiles leave a split-K second round).  Four waves
// side by side along N, each owning BN/4 rows of B^T, which it loads from HBM
// straight into its MFMA fragment registers four k-steps ahead (no two waves
// read the same B row); A is shared through a ring of four LDS stages, its
// loads issued two stages before they are stored.  One k-step (32 k) per
// stage, v_mfma_f32_16x16x32_{bf16,f16}: lane (l16, q) holds row l16 of a
// 16-row block, k = 8 q .. 8 q + 7; accumulator item r is row 4 q + r,
// column l16.
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));

template <bool BF>
__device__ __forceinline__ v4f mfma16x16(u4 a, u4 b, v4f c) {
  if constexpr (BF)
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a),
                                                  __builtin_bit_cast(v8h, b), c, 0, 0, 0);
}

// One k-step of MB x NB blocks; nb holds -Im B (sign bits flipped).  Each
// accumulator takes its products in the order of mma_ab: per term pair
// (small terms first) real part Ar Br then -Ai Bi, imaginary part Ar Bi then
// Ai Br; consecutive MFMAs go to different accumulators.
template <int MB, int NB, bool BF, int NT>
__device__ __forceinline__ void mma16(const u4 (&fa)[MB][2 * NT], const u4 (&fb)[NB][2 * NT],
                                      v4f (&accR)[MB][NB], v4f (&accI)[MB][NB]) {
  u4 nb[NB][NT];
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int t = 0; t < NT; ++t) nb[j][t] = fb[j][NT + t] ^ 0x80008000u;
#pragma unroll
  for (int s = NT - 1; s >= 0; --s)
#pragma unroll
    for (int ta = 0; ta <= s; ++ta) {
      const int tb = s - ta;
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          accR[i][j] = mfma16x16<BF>(fa[i][ta], fb[j][tb], accR[i][j]);
          accI[i][j] = mfma16x16<BF>(fa[i][ta], fb[j][NT + tb], accI[i][j]);
        }
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          accR[i][j] = mfma16x16<BF>(fa[i][NT + ta], nb[j][tb], accR[i][j]);
          accI[i][j] = mfma16x16<BF>(fa[i][NT + ta], fb[j][tb], accI[i][j]);
        }
    }
}

template <int BM, int BN, int NT, int EPI>
constexpr int d16_lds_bytes() {
  constexpr int ring = 4 * 2 * NT * BM * 4 * 16;              // four A stages
  constexpr int tr = EPI == EPI_PROJECT  ? 2 * NT * BN * (BM + 8) * 2
                     : EPI == EPI_GATHER ? gather_lds_bytes<BM, BN>()
                                         : 0;
  return ring > tr ? ring : tr;
}

// Tile of schedule rank r with the ranks laid out in gm groups along M: group
// g holds the M tiles g tiles_m / gm .. (g + 1) tiles_m / gm - 1 of every N
// tile, M fastest, so that the ranks an XCD runs (one contiguous range of
// them) read about 1/gm of A and a band of B instead of all of A.
__device__ __forceinline__ int rank_tile(int r, int tiles_m, int tiles, int gm) {
  if (gm <= 1 || tiles_m % gm) return r;
  const int G = tiles / gm, tm = tiles_m / gm;
  const int g = r / G, w = r % G;
  return (w / tm) * tiles_m + g * tm + w % tm;
}

// The main loop over all of K; false when the done flag stops the product.
template <int BM, int BN, bool BF, int NT, bool PRE>
__device__ __forceinline__ bool d16_loop(const SplitArgs &a, int m0, int n0, int tid, u4 *lds,
                                         v4f (&accR)[BM / 16][BN / 64],
                                         v4f (&accI)[BM / 16][BN / 64], GatherPre &gp) {
  constexpr int WTN = BN / 4, MB = BM / 16, NB = WTN / 16, PL = 2 * NT, CH = 4;
  constexpr int LA = PL * BM * CH, NA = LA / kThreads, SA = LA;
  static_assert(LA % kThreads == 0 && WTN % 16 == 0 && BM % 16 == 0, "d16 tile");
  const int lane = tid & 63, wave = tid >> 6, l16 = lane & 15, q = lane >> 4;
  const unsigned short *ga[NA];
  int la[NA];
#pragma unroll
  for (int s_ = 0; s_ < NA; ++s_) {
    const int id = tid + kThreads * s_;
    const int c = id % CH, row = (id / CH) % BM, plane = id / (CH * BM);
    ga[s_] = a.a + (size_t)plane * a.a_plane + (size_t)(m0 + row) * kKB + 8 * c;
    la[s_] = (plane * BM + row) * CH + c;
  }
  // B^T row of lane (l16, q) in block j: n0 + WTN wave + 16 j + l16, k 8q .. 8q + 7
  const unsigned short *gb = a.b + (size_t)(n0 + WTN * wave + l16) * kKB + 8 * q;
  const int KT = a.K / kKB;
  if (KT <= 0) return !(a.done && *a.done);
  const int last = KT - 1;
  u4 ra0[NA], ra1[NA];
  u4 bq0[NB][PL], bq1[NB][PL], bq2[NB][PL], bq3[NB][PL];
#define E_LOAD_A(RA, KT_)                                                                 \
  do {                                                                                    \
    const size_t o_ = (size_t)(KT_) * a.M * kKB;                                          \
    _Pragma("unroll") for (int s_ = 0; s_ < NA; ++s_) RA[s_] =                            \
        *reinterpret_cast<const u4 *>(ga[s_] + o_);                                       \
  } while (0)
#define E_LOAD_B(BQ, KT_)                                                                 \
  do {                                                                                    \
    const size_t o_ = (size_t)(KT_) * a.N * kKB;                                          \
    _Pragma("unroll") for (int j_ = 0; j_ < NB; ++j_)                                     \
        _Pragma("unroll") for (int p_ = 0; p_ < PL; ++p_) BQ[j_][p_] =                    \
            *reinterpret_cast<const u4 *>(gb + p_ * a.b_plane + (size_t)16 * j_ * kKB + o_); \
  } while (0)
#define E_STORE_A(RA, BUF)                                                                \
  do {                                                                                    \
    _Pragma("unroll") for (int s_ = 0; s_ < NA; ++s_) lds[(BUF) * SA + la[s_]] = RA[s_];  \
  } while (0)
#define E_READ_A(F, BUF)                                                                  \
  do {                                                                                    \
    _Pragma("unroll") for (int i_ = 0; i_ < MB; ++i_)                                     \
        _Pragma("unroll") for (int p_ = 0; p_ < PL; ++p_) F[i_][p_] =                     \
            lds[(BUF) * SA + (p_ * BM + 16 * i_ + l16) * CH + q];                         \
  } while (0)
  // Prologue.  The loads still in flight when the loop starts are issued in
  // the order a loop step issues them (A of stage 2, its B, A of stage 3,
  // its B), so that the wait counts the compiler sets at the top of the loop,
  // which must hold for the first iteration as for every later one, are the
  // steady-state ones and do not drain the prefetch on each iteration.
  E_LOAD_A(ra0, 0);
  E_LOAD_A(ra1, 1 < last ? 1 : last);
  E_LOAD_B(bq0, 0);
  E_LOAD_B(bq1, 1 < last ? 1 : last);
  if constexpr (PRE) gather_pre_foci(a.g, m0, tid, gp);   // behind the operand loads
  const int stop = a.done ? *a.done : 0;
  asm volatile("" ::: "memory");
  if (stop) return false;
  E_STORE_A(ra0, 0);
  E_STORE_A(ra1, 1);
  __builtin_amdgcn_sched_barrier(0);
  E_LOAD_A(ra0, 2 < last ? 2 : last);
  E_LOAD_B(bq2, 2 < last ? 2 : last);
  __builtin_amdgcn_sched_barrier(0);
  E_LOAD_A(ra1, 3 < last ? 3 : last);
  E_LOAD_B(bq3, 3 < last ? 3 : last);
  __builtin_amdgcn_sched_barrier(0);
  __syncthreads();
  u4 f0[MB][PL], f1[MB][PL];
  E_READ_A(f0, 0);
  // per step: NR fragment reads, NM MFMAs, NA stores, NV loads
  constexpr int NR = MB * PL, NM = MB * NB * 2 * NT * (NT + 1), NV = NA + NB * PL;
  static_assert(NM >= NR + NA + NV, "interleave pattern");
  // Step s (stage s in LDS buffer s & 3, its A fragments in FA, its B in
  // BQ): read stage s + 1's A fragments into FB while the MFMAs run, store
  // stage s + 2 (in registers since two steps ago) into buffer (s + 2) & 3,
  // issue the loads of stage s + 4 of A and B, one barrier.
#define E_STEP(S, FA, FB, RA, BQ, B1, B2)                                                 \
  do {                                                                                    \
    E_READ_A(FB, B1);                                                                     \
    mma16<MB, NB, BF, NT>(FA, BQ, accR, accI);                                            \
    E_STORE_A(RA, B2);                                                                    \
    E_LOAD_A(RA, (S) + 4 < last ? (S) + 4 : last);                                        \
    E_LOAD_B(BQ, (S) + 4 < last ? (S) + 4 : last);                                        \
    sched_read_mfma<NR>();                                                                \
    sched_write_mfma<NA, 1>();                                                            \
    sched_vmem_mfma<NV>();                                                                \
    __builtin_amdgcn_sched_group_barrier(0x008, NM - NR - NA - NV, 0);                    \
    __builtin_amdgcn_sched_barrier(0);                                                    \
    __syncthreads();                                                                      \
  } while (0)
  int s = 0;
  for (; s + 3 < KT; s += 4) {
    E_STEP(s, f0, f1, ra0, bq0, 1, 2);
    E_STEP(s + 1, f1, f0, ra1, bq1, 2, 3);
    E_STEP(s + 2, f0, f1, ra0, bq2, 3, 0);
    E_STEP(s + 3, f1, f0, ra1, bq3, 0, 1);
  }
  if (s < KT) E_STEP(s, f0, f1, ra0, bq0, 1, 2);
  if (s + 1 < KT) E_STEP(s + 1, f1, f0, ra1, bq1, 2, 3);
  if (s + 2 < KT) E_STEP(s + 2, f0, f1, ra0, bq2, 3, 0);
#undef E_STEP
#undef E_LOAD_A
#undef E_LOAD_B
#undef E_STORE_A
#undef E_READ_A
  return true;
}

// One whole tile per workgroup (no K split); epilogues: store float32 C, or
// project onto the amplitude constraint and write the split planes of P^T.
template <int BM, int BN, bool BF, int NT, int EPI>
__device__ __forceinline__ void cgemm_split_d16_unit(const SplitArgs &a, const int t,
                                                     const int prow, u4 *lds) {
  constexpr int WTN = BN / 4, MB = BM / 16, NB = WTN / 16, PL = 2 * NT, TP = BM + 8;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, q = lane >> 4;
  const int m0 = (t % a.tiles_m) * BM, n0 = (t / a.tiles_m) * BN;
  v4f accR[MB][NB], accI[MB][NB];
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      accR[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
      accI[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  // the gather's focus indices: row range now, foci behind the operand loads
  GatherPre gp;
  if constexpr (EPI == EPI_GATHER) gather_pre_rows(a.g, m0, BM, gp);
  if (!d16_loop<BM, BN, BF, NT, EPI == EPI_GATHER>(a, m0, n0, tid, lds, accR, accI, gp)) return;
  if constexpr (EPI == EPI_GATHER) {
    // stage the tile of L in LDS, then gather the tile's foci from it
    constexpr int LD = BN + 1;
    float *tr = reinterpret_cast<float *>(lds), *ti = tr + BM * LD;
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ml = 16 * i + 4 * q + r, nl = wave * WTN + 16 * j + l16;
          tr[ml * LD + nl] = accR[i][j][r];
          ti[ml * LD + nl] = accI[i][j][r];
        }
    __syncthreads();
    gather_tile_lds<BM, BN>(a.g, reinterpret_cast<float *>(lds), m0, n0, tid, gp,
                            prow >= 0 ? prow : n0 / BN);
  } else if constexpr (EPI == EPI_STORE) {
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int n = n0 + wave * WTN + 16 * j + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const size_t o = (size_t)(m0 + 16 * i + 4 * q + r) * a.ldc + n;
          a.cr[o] = accR[i][j][r];
          a.ci[o] = accI[i][j][r];
        }
      }
  } else if constexpr (EPI == EPI_PROJECT) {
    // the projection's amplitudes, read after the main loop (held through it
    // they would add to its register pressure)
    float ampv[MB][NB][4];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          ampv[i][j][r] = a.amp[(size_t)(m0 + 16 * i + 4 * q + r) * a.ldc + n0 + wave * WTN +
                                16 * j + l16];
    // project, split into terms, transpose the tile through LDS, then write
    // rows of P^T [plane][n][m0 .. m0 + BM) in 16-byte runs
    unsigned short *tt = reinterpret_cast<unsigned short *>(lds);
    __syncthreads();   // operand stages are no longer read
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int nl = wave * WTN + 16 * j + l16, ml = 16 * i + 4 * q;
        unsigned short tr[NT][4], ti[NT][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float pr, pi;
          project_amp(accR[i][j][r], accI[i][j][r], ampv[i][j][r], pr, pi);
          split_terms<BF, NT>(pr, &tr[0][r], 4);
          split_terms<BF, NT>(pi, &ti[0][r], 4);
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          const u2 vr = {(unsigned)tr[u][0] | ((unsigned)tr[u][1] << 16),
                         (unsigned)tr[u][2] | ((unsigned)tr[u][3] << 16)};
          const u2 vi = {(unsigned)ti[u][0] | ((unsigned)ti[u][1] << 16),
                         (unsigned)ti[u][2] | ((unsigned)ti[u][3] << 16)};
          *reinterpret_cast<u2 *>(tt + ((size_t)u * BN + nl) * TP + ml) = vr;
          *reinterpret_cast<u2 *>(tt + ((size_t)(NT + u) * BN + nl) * TP + ml) = vi;
        }
      }
    __syncthreads();
    constexpr int RC = BM / 8;                  // 16-byte chunks per row
    constexpr int NCH = PL * BN * RC;
    static_assert(NCH % kThreads == 0, "epilogue chunking");
#pragma unroll
    for (int s_ = 0; s_ < NCH / kThreads; ++s_) {
      const int id = tid + kThreads * s_;
      const int c = id % RC, nl = (id / RC) % BN, pl = id / (RC * BN);
      const u4 v = *reinterpret_cast<const u4 *>(tt + ((size_t)pl * BN + nl) * TP + 8 * c);
      *reinterpret_cast<u4 *>(a.pt + (size_t)pl * a.pt_plane +
                              kblk_index(n0 + nl, m0 + 8 * c, a.N)) = v;   // 8 m, one k-block
    }
  }
}

template <int BM, int BN, bool BF, int NT, int EPI>
__global__ __launch_bounds__(kThreads) void cgemm_split_d16(SplitArgs a) {
  __shared__ u4 lds[(d16_lds_bytes<BM, BN, NT, EPI>() + 15) / 16];
  const int t = rank_tile(xcd_tile(blockIdx.x, a.t_dp), a.tiles_m, a.t_dp, a.xgm);
  cgemm_split_d16_unit<BM, BN, BF, NT, EPI>(a, t, -1, lds);
}

// Work-list launch of the 16x16-block loop (whole K per unit).
template <int BM, int BN, bool BF, int NT, int EPI>
__global__ __launch_bounds__(kThreads) void cgemm_split_d16_work(const SplitArgs *items,
                                                                 const WorkUnit *work,
                                                                 const int *off, int n) {
  __shared__ u4 lds[(d16_lds_bytes<BM, BN, NT, EPI>() + 15) / 16];
  // units off[b] .. off[b + 1] - 1 (persistent), or unit b (off null)
  const int w0 = off ? off[blockIdx.x] : (int)blockIdx.x;
  const int w1 = off ? off[blockIdx.x + 1] : w0 + 1;
  for (int w = w0; w < w1 && w < n; ++w) {
    if (w != w0) __syncthreads();   // the previous unit's LDS reads are done
    const WorkUnit u = work[w];
    cgemm_split_d16_unit<BM, BN, BF, NT, EPI>(items[u.item], u.tile, u.prow, lds);
  }
}

template <bool BF, int NT, int EPI>
hipError_t launch_d16(const GemmTile &tl, const SplitArgs &args, int grid, hipStream_t s) {
  if constexpr (NT == 2) {
    if constexpr (EPI == EPI_PROJECT || EPI == EPI_STORE) {
      if (tl.bm == 48 && tl.bn == 192) {
        hipLaunchKernelGGL((cgemm_split_d16<48, 192, BF, NT, EPI>), dim3(grid), dim3(kThreads),
                           0, s, args);
        return hipGetLastError();
      }
    }
    if constexpr (EPI == EPI_GATHER) {
      if (tl.bm == 64 && tl.bn == 128) {
        hipLaunchKernelGGL((cgemm_split_d16<64, 128, BF, NT, EPI>), dim3(grid), dim3(kThreads),
                           0, s, args);
        return hipGetLastError();
      }
    }
  }
  return hipErrorInvalidValue;
}

template <int BM, int BN, int BK, bool BF, int NT, int EPI, int KG, int PIPE>
hipError_t launch_t(const SplitArgs &args, int grid, hipStream_t s) {
  hipLaunchKernelGGL((cgemm_split_mfma<BM, BN, BK, BF, NT, EPI, KG, PIPE>), dim3(grid),
                     dim3(kThreads * KG), 0, s, args);
  return hipGetLastError();
}

template <int BM, int BN, int BK, bool BF, int NT, int EPI, int KG = 1, int PIPE = 0>
hipError_t launch_fit(const SplitArgs &args, int grid, hipStream_t s) {
  if constexpr (split_lds_bytes<BM, BN, BK, NT, EPI, PIPE>() <= 160 * 1024)
    return launch_t<BM, BN, BK, BF, NT, EPI, KG, PIPE>(args, grid, s);
  return hipErrorInvalidValue;
}

template <bool BF, int NT>
hipError_t launch_tail_t(const GemmTile &tl, const SplitArgs &a, int n_tail, hipStream_t s) {
  const dim3 g(n_tail, 4);
#define TAIL(BM, BN, COLS) \
  hipLaunchKernelGGL((cgemm_tail_project_split<BM, BN, BF, NT, COLS>), g, dim3(kThreads), 0, s, a)
  if (tl.pipe == 2 && tl.bm == 64 && tl.bn == 128) TAIL(64, 128, true);
  else if (tl.bm == 64 && tl.bn == 64) TAIL(64, 64, false);
  else if (tl.bm == 64 && tl.bn == 128) TAIL(64, 128, false);
  else if (tl.bm == 128 && tl.bn == 64) TAIL(128, 64, false);
  else if (tl.bm == 128 && tl.bn == 128) TAIL(128, 128, false);
  else return hipErrorInvalidValue;
#undef TAIL
  return hipGetLastError();
}

hipError_t launch_tail_split(int precision, const GemmTile &tl, const SplitArgs &a, int n_tail,
                             hipStream_t s) {
  switch (precision) {
    case GSWMTP_BF16X3: return launch_tail_t<true, 2>(tl, a, n_tail, s);
    case GSWMTP_FP16X3: return launch_tail_t<false, 2>(tl, a, n_tail, s);
    case GSWMTP_BF16X6: return launch_tail_t<true, 3>(tl, a, n_tail, s);
  }
  return hipErrorInvalidValue;
}

template <bool BF, int NT, int EPI>
hipError_t launch_e(const GemmTile &tl, const SplitArgs &args, int grid, hipStream_t s) {
  if (tl.pipe == 3) return launch_d16<BF, NT, EPI>(tl, args, grid, s);
  if (tl.bk == 32) {
    if (tl.bm == 64 && tl.bn == 64) {
      if (tl.pipe) return launch_fit<64, 64, 32, BF, NT, EPI, 1, 1>(args, grid, s);
      return tl.kg == 2 ? launch_fit<64, 64, 32, BF, NT, EPI, 2>(args, grid, s)
                        : launch_fit<64, 64, 32, BF, NT, EPI>(args, grid, s);
    }
    if (tl.bm == 128 && tl.bn == 64)
      return tl.pipe ? launch_fit<128, 64, 32, BF, NT, EPI, 1, 1>(args, grid, s)
                     : launch_fit<128, 64, 32, BF, NT, EPI>(args, grid, s);
    if (tl.bm == 64 && tl.bn == 128) {
      if constexpr (NT == 2)
        if (tl.pipe == 2) return launch_fit<64, 128, 32, BF, NT, EPI, 1, 2>(args, grid, s);
      return tl.pipe ? launch_fit<64, 128, 32, BF, NT, EPI, 1, 1>(args, grid, s)
                     : launch_fit<64, 128, 32, BF, NT, EPI>(args, grid, s);
    }
    if (tl.bm == 128 && tl.bn == 128) return launch_fit<128, 128, 32, BF, NT, EPI>(args, grid, s);
  } else if (tl.bk == 16) {
    if (tl.bm == 64 && tl.bn == 64) return launch_fit<64, 64, 16, BF, NT, EPI>(args, grid, s);
    if (tl.bm == 128 && tl.bn == 64) return launch_fit<128, 64, 16, BF, NT, EPI>(args, grid, s);
    if (tl.bm == 64 && tl.bn == 128) return launch_fit<64, 128, 16, BF, NT, EPI>(args, grid, s);
    if (tl.bm == 128 && tl.bn == 128) return launch_fit<128, 128, 16, BF, NT, EPI>(args, grid, s);
  }
  return hipErrorInvalidValue;
}

template <int EPI>
hipError_t launch_p(int precision, const GemmTile &tl, const SplitArgs &args, int grid,
                    hipStream_t s) {
  switch (precision) {
    case GSWMTP_BF16X3: return launch_e<true, 2, EPI>(tl, args, grid, s);
    case GSWMTP_FP16X3: return launch_e<false, 2, EPI>(tl, args, grid, s);
    case GSWMTP_BF16X6: return launch_e<true, 3, EPI>(tl, args, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

namespace {

// Operand, output and epilogue pointers of one plan's split product.
SplitArgs split_args(const gswmtp_plan *p, bool forward, const unsigned short *bt, float *cr,
                     float *ci, unsigned short *pt_out, bool honour_done) {
  const Dims &d = p->d;
  SplitArgs a{};
  if (forward) {
    a.a = p->b.as_f;
    a.M = d.Urp;
    a.K = d.Rp;
  } else {
    a.a = p->b.as_b;
    a.M = d.Rp;
    a.K = d.Urp;
  }
  a.N = d.Cp;
  a.a_plane = (size_t)a.M * a.K;
  a.b = bt;
  a.b_plane = (size_t)a.N * a.K;
  a.cr = cr;
  a.ci = ci;
  a.ldc = d.Cp;
  a.amp = p->b.amp;
  a.pt = pt_out;
  a.pt_plane = (size_t)d.Cp * d.Rp;
  a.done = honour_done ? p->b.ctrl + CTRL_DONE : nullptr;
  a.part = p->b.part;
  a.g = gather_ctx(p);
  return a;
}

}  // namespace

hipError_t launch_cgemm_split(const gswmtp_plan *p, bool forward, int epi,
                              const unsigned short *bt, float *cr, float *ci,
                              unsigned short *pt_out, bool honour_done, hipStream_t s,
                              int phases, const unsigned short *at) {
  const GemmSched &sc = forward ? p->sched_fwd : p->sched_bwd;
  const int nt = split_terms_of(p->precision);
  SplitArgs a = split_args(p, forward, bt, cr, ci, pt_out, honour_done);
  if (at) a.a = at;   // same shape and layout as the default left operand
  if (nt < 2 || a.M % sc.tile.bm || a.N % sc.tile.bn || a.K % sc.tile.bk)
    return hipErrorInvalidValue;
  if (sc.tiles_m * sc.tile.bm != a.M || sc.tiles * sc.tile.bm * sc.tile.bn != a.M * a.N)
    return hipErrorInvalidValue;
  if (epi != EPI_STORE && epi != EPI_PROJECT && epi != EPI_GATHER) return hipErrorInvalidValue;
  if (epi == EPI_PROJECT && (forward || !pt_out)) return hipErrorInvalidValue;
  if (epi == EPI_GATHER && !forward) return hipErrorInvalidValue;
  a.tiles_m = sc.tiles_m;
  a.t_dp = sc.t_dp;
  a.split = sc.split;
  a.xgm = sc.xgm;
  if (sc.tile.pipe == 3 && sc.n_tail > 0) return hipErrorInvalidValue;
  for (int phase = 0; phase < (sc.n_tail > 0 ? 2 : 1); ++phase) {
    if (!(phases & (1 << phase))) continue;
    a.phase = phase;
    const int grid = phase == 0 ? sc.grid : sc.n_tail;
    if (phase == 1 && epi == EPI_PROJECT) {
      const hipError_t e = launch_tail_split(p->precision, sc.tile, a, sc.n_tail, s);
      if (e != hipSuccess) return e;
      continue;
    }
    const hipError_t e = epi == EPI_STORE    ? launch_p<EPI_STORE>(p->precision, sc.tile, a, grid, s)
                         : epi == EPI_GATHER ? launch_p<EPI_GATHER>(p->precision, sc.tile, a, grid, s)
                                             : launch_p<EPI_PROJECT>(p->precision, sc.tile, a, grid, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}


// A split product with explicit operands, both stored as 16-bit term planes
// of [rows][K] matrices, k-blocked: C[M][N] = sum_k A[m][k] B[n][k] into
// float32 planes cr / ci [M][ldc], on schedule sc (the grid form's first
// product, L^T = P^T Omega_r^T).
hipError_t launch_cgemm_split_ex(const gswmtp_plan *p, const GemmSched &sc,
                                 const unsigned short *a, int M, const unsigned short *b, int N,
                                 int K, float *cr, float *ci, int ldc, bool honour_done,
                                 hipStream_t s) {
  const int nt = split_terms_of(p->precision);
  if (nt < 2 || sc.tile.pipe == 3 || M % sc.tile.bm || N % sc.tile.bn || K % sc.tile.bk ||
      sc.tiles_m * sc.tile.bm != M || sc.tiles * sc.tile.bm * sc.tile.bn != M * N)
    return hipErrorInvalidValue;
  SplitArgs x{};
  x.a = a;
  x.M = M;
  x.K = K;
  x.a_plane = (size_t)M * K;
  x.b = b;
  x.N = N;
  x.b_plane = (size_t)N * K;
  x.cr = cr;
  x.ci = ci;
  x.ldc = ldc;
  x.done = honour_done ? p->b.ctrl + CTRL_DONE : nullptr;
  x.part = p->b.part;
  x.tiles_m = sc.tiles_m;
  x.t_dp = sc.t_dp;
  x.split = sc.split;
  x.xgm = sc.xgm;
  for (int phase = 0; phase < (sc.n_tail > 0 ? 2 : 1); ++phase) {
    x.phase = phase;
    const hipError_t e =
        launch_p<EPI_STORE>(p->precision, sc.tile, x, phase == 0 ? sc.grid : sc.n_tail, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

namespace {

// Float32 planes S [Urp][ldc] as the split planes of S^T ([2][NT] x [Cp][Urp],
// k-blocked), times an exact power-of-two scale: one (c, u) per thread, u
// fastest so every store run is contiguous.
template <bool BF, int NT>
__global__ void k_split_transpose(const float *__restrict__ sr, const float *__restrict__ si,
                                  int Urp, int Cp, int ldc, float scale,
                                  unsigned short *__restrict__ st, const int *done) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)Urp * Cp) return;
  const int u = (int)(id % Urp), c = (int)(id / Urp);
  const float re = sr[(size_t)u * ldc + c] * scale, im = si[(size_t)u * ldc + c] * scale;
  if (done && *done) return;
  const size_t plane = (size_t)Cp * Urp, at = kblk_index(c, u, Cp);
  split_terms<BF, NT>(re, st + at, (int)plane);
  split_terms<BF, NT>(im, st + (size_t)NT * plane + at, (int)plane);
}

}  // namespace

hipError_t launch_split_transpose(const gswmtp_plan *p, const float *sr, const float *si,
                                  float scale, bool honour_done, hipStream_t s) {
  const Dims &d = p->d;
  const dim3 grid((unsigned)(((size_t)d.Urp * d.Cp + 255) / 256));
  const int *done = honour_done ? p->b.ctrl + CTRL_DONE : nullptr;
#define SPLIT_T(BF, NT)                                                                       \
  hipLaunchKernelGGL((k_split_transpose<BF, NT>), grid, dim3(256), 0, s, sr, si, d.Urp, d.Cp, \
                     d.Cp, scale, p->b.ss, done)
  switch (p->precision) {
    case GSWMTP_BF16X3: SPLIT_T(true, 2); break;
    case GSWMTP_FP16X3: SPLIT_T(false, 2); break;
    case GSWMTP_BF16X6: SPLIT_T(true, 3); break;
    default: return hipErrorInvalidValue;
  }
#undef SPLIT_T
  return hipGetLastError();
}

// ---- batched form: work-list launches ----------------------------------------

size_t split_args_bytes() { return sizeof(SplitArgs); }

int fill_split_args(const gswmtp_plan *p, bool forward, const GemmTile &tl, bool honour_done,
                    unsigned short *pt_out, void *out) {
  SplitArgs a = forward ? split_args(p, true, p->b.ps, nullptr, nullptr, nullptr, honour_done)
                        : split_args(p, false, p->scaled_adj ? p->b.bs : p->b.ss, nullptr,
                                     nullptr, pt_out ? pt_out : p->b.ps, honour_done);
  if (!forward && p->scaled_adj) a.a = p->b.as_s;   // the re-associated adjoint
  a.tiles_m = a.M / tl.bm;
  a.t_dp = a.tiles_m * (a.N / tl.bn);
  a.split = 1;
  a.phase = 0;
  std::memcpy(out, &a, sizeof a);
  return a.t_dp;
}

namespace {

template <int BM, int BN, bool BF, int NT, int EPI, int KG, int PIPE>
hipError_t work_t(const WorkLaunch &w, hipStream_t s, int *occ) {
  if constexpr (split_lds_bytes<BM, BN, 32, NT, EPI, PIPE>() <= 160 * 1024) {
    if (occ)
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(
          occ, cgemm_split_work<BM, BN, 32, BF, NT, EPI, KG, PIPE>, kThreads * KG, 0);
    // k-group loops end group 1 early in each unit, so a unit per workgroup
    // (the loop in the kernel runs once): no barrier after a unit
    const int grid = KG > 1 ? w.n_work : w.grid;
    hipLaunchKernelGGL((cgemm_split_work<BM, BN, 32, BF, NT, EPI, KG, PIPE>), dim3(grid),
                       dim3(kThreads * KG), 0, s, static_cast<const SplitArgs *>(w.d_items),
                       w.d_work, KG > 1 ? nullptr : w.d_off, w.n_work);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <int BM, int BN, bool BF, int NT, int EPI>
hipError_t work_d16_t(const WorkLaunch &w, hipStream_t s, int *occ) {
  if (occ)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        occ, cgemm_split_d16_work<BM, BN, BF, NT, EPI>, kThreads, 0);
  hipLaunchKernelGGL((cgemm_split_d16_work<BM, BN, BF, NT, EPI>), dim3(w.grid), dim3(kThreads), 0,
                     s, static_cast<const SplitArgs *>(w.d_items), w.d_work, w.d_off, w.n_work);
  return hipGetLastError();
}

// occ != null: only report the kernel's resident workgroups per CU
template <bool BF, int NT, int EPI>
hipError_t work_e(const WorkLaunch &w, hipStream_t s, int *occ) {
  const GemmTile &t = w.cfg.tile;
  if constexpr (NT == 2) {
    if (t.pipe == 3) {
      if constexpr (EPI == EPI_PROJECT)
        if (t.bm == 48 && t.bn == 192) return work_d16_t<48, 192, BF, NT, EPI>(w, s, occ);
      if constexpr (EPI == EPI_GATHER)
        if (t.bm == 64 && t.bn == 128) return work_d16_t<64, 128, BF, NT, EPI>(w, s, occ);
      if (t.bm == 64 && t.bn == 64) return work_d16_t<64, 64, BF, NT, EPI>(w, s, occ);
      return hipErrorInvalidValue;
    }
    if (t.bk != 32 || t.bm != 64) return hipErrorInvalidValue;
    if (t.pipe == 1 && t.bn == 64) return work_t<64, 64, BF, NT, EPI, 1, 1>(w, s, occ);
    if (t.pipe == 1 && t.bn == 128) return work_t<64, 128, BF, NT, EPI, 1, 1>(w, s, occ);
    if (t.pipe == 2 && t.bn == 128) return work_t<64, 128, BF, NT, EPI, 1, 2>(w, s, occ);
  } else {
    if (t.bk == 32 && t.bm == 64 && t.bn == 64 && t.kg == 2)
      return work_t<64, 64, BF, NT, EPI, 2, 0>(w, s, occ);
  }
  return hipErrorInvalidValue;
}

template <int EPI>
hipError_t work_p(int precision, const WorkLaunch &w, hipStream_t s, int *occ) {
  switch (precision) {
    case GSWMTP_BF16X3: return work_e<true, 2, EPI>(w, s, occ);
    case GSWMTP_FP16X3: return work_e<false, 2, EPI>(w, s, occ);
    case GSWMTP_BF16X6: return work_e<true, 3, EPI>(w, s, occ);
  }
  return hipErrorInvalidValue;
}

hipError_t work_dispatch(const WorkLaunch &w, hipStream_t s, int *occ) {
  if (w.epi == EPI_GATHER) return work_p<EPI_GATHER>(w.precision, w, s, occ);
  if (w.epi == EPI_PROJECT) return work_p<EPI_PROJECT>(w.precision, w, s, occ);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_cgemm_split_work(const WorkLaunch &w, hipStream_t s) {
  if (w.n_work == 0) return hipSuccess;
  return work_dispatch(w, s, nullptr);
}

int cgemm_split_work_occupancy(const WorkConfig &c, int epi, int precision) {
  WorkLaunch w;
  w.cfg = c;
  w.epi = epi;
  w.precision = precision;
  int n = 0;
  return work_dispatch(w, nullptr, &n) == hipSuccess ? n : 0;
}

}  // namespace gswmtp
