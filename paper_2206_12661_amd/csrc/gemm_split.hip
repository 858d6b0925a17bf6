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
// Layout: both operands k-contiguous, 16-bit planes [re/im][term][row][K]:
//   forward   A = Omega_r [Urp][Rp],      B^T = P^T [Cp][Rp]
//   adjoint   A = Omega_r^H [Rp][Urp],    B^T = S^T [Cp][Urp]
// so each MFMA operand fragment (8 consecutive k of one row) is one 16-byte
// LDS read.  LDS rows hold 16 k (two 16-byte chunks); the chunk index is
// XOR-swizzled with row bits 2 and 3 so fragment reads of 8 or 16 lanes hit
// distinct banks.
//
// Scheduling, split-K tail and in-order reduction as in the float32 kernel.
// Epilogues: store float32 C (forward, for the focus gather); or project onto
// the amplitude constraint and write the pupil field directly as the split
// B^T planes of the next forward product.
#include "gswmtp_internal.h"

namespace gswmtp {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int kBK = 16;

template <bool BF>
__device__ __forceinline__ v16f mfma16(u4 a, u4 b, v16f c) {
  if constexpr (BF)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a),
                                                  __builtin_bit_cast(v8h, b), c, 0, 0, 0);
}

__device__ __forceinline__ int xcd_tile(int bid, int tiles) {
  const int xcd = bid & 7, local = bid >> 3;
  const int per = tiles >> 3, rem = tiles & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + local;
}

__device__ __forceinline__ int swz(int row) { return ((row >> 2) ^ (row >> 3)) & 1; }

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
  int *cnt;
  int tiles_m, t_dp, split;
};

template <int BM, int BN, bool BF, int NT, int EPI>
__global__ __launch_bounds__(kThreads) void cgemm_split_mfma(SplitArgs a) {
  if (a.done && *a.done) return;
  constexpr int WTM = BM / 2, WTN = BN / 2;
  constexpr int MB = WTM / 32, NB = WTN / 32;
  constexpr int PL = 2 * NT;                     // planes per operand
  constexpr int LA = PL * BM * 2, LB = PL * BN * 2;   // 16-byte chunks per stage
  constexpr int NA = LA / kThreads, NBL = LB / kThreads;
  static_assert(LA % kThreads == 0 && LB % kThreads == 0, "tile/thread mismatch");

  __shared__ u4 sA[2][LA];
  __shared__ u4 sB[2][LB];
  __shared__ int s_last;

  const int tid = threadIdx.x;
  const int KT = a.K / kBK;
  int t, kb, ke, tail = -1, chunk = 0;
  if ((int)blockIdx.x < a.t_dp) {
    t = xcd_tile(blockIdx.x, a.t_dp);
    kb = 0;
    ke = KT;
  } else {
    const int u = blockIdx.x - a.t_dp;
    tail = u / a.split;
    chunk = u % a.split;
    t = a.t_dp + tail;
    kb = chunk * KT / a.split;
    ke = (chunk + 1) * KT / a.split;
  }
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

  // staging: chunk id = (plane * rows + row) * 2 + c (16 bytes, 8 k values)
  const unsigned short *ga[NA];
  const unsigned short *gb[NBL];
  int la[NA], lb[NBL];
#pragma unroll
  for (int s = 0; s < NA; ++s) {
    const int id = tid + kThreads * s;
    const int c = id & 1, row = (id >> 1) % BM, plane = (id >> 1) / BM;
    ga[s] = a.a + (size_t)plane * a.a_plane + (size_t)(m0 + row) * a.K + 8 * c;
    la[s] = (plane * BM + row) * 2 + (c ^ swz(row));
  }
#pragma unroll
  for (int s = 0; s < NBL; ++s) {
    const int id = tid + kThreads * s;
    const int c = id & 1, row = (id >> 1) % BN, plane = (id >> 1) / BN;
    gb[s] = a.b + (size_t)plane * a.b_plane + (size_t)(n0 + row) * a.K + 8 * c;
    lb[s] = (plane * BN + row) * 2 + (c ^ swz(row));
  }
  u4 ra[NA], rb[NBL];
  if (kb < ke) {
#pragma unroll
    for (int s = 0; s < NA; ++s) ra[s] = *reinterpret_cast<const u4 *>(ga[s] + kb * kBK);
#pragma unroll
    for (int s = 0; s < NBL; ++s) rb[s] = *reinterpret_cast<const u4 *>(gb[s] + kb * kBK);
#pragma unroll
    for (int s = 0; s < NA; ++s) sA[0][la[s]] = ra[s];
#pragma unroll
    for (int s = 0; s < NBL; ++s) sB[0][lb[s]] = rb[s];
  }
  __syncthreads();

  for (int kt = kb; kt < ke; ++kt) {
    const int buf = (kt - kb) & 1;
    const bool more = kt + 1 < ke;
    if (more) {
#pragma unroll
      for (int s = 0; s < NA; ++s)
        ra[s] = *reinterpret_cast<const u4 *>(ga[s] + (kt + 1) * kBK);
#pragma unroll
      for (int s = 0; s < NBL; ++s)
        rb[s] = *reinterpret_cast<const u4 *>(gb[s] + (kt + 1) * kBK);
    }
    // fragments: lane (l32, h) reads row l32 of its block, k = 8h .. 8h + 7
    u4 fa[MB][PL], fb[NB][PL], na[MB][NT];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const int row = wm * WTM + i * 32 + l32;
#pragma unroll
      for (int pl = 0; pl < PL; ++pl) fa[i][pl] = sA[buf][(pl * BM + row) * 2 + (h ^ swz(row))];
#pragma unroll
      for (int q = 0; q < NT; ++q) na[i][q] = fa[i][NT + q] ^ 0x80008000u;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int row = wn * WTN + j * 32 + l32;
#pragma unroll
      for (int pl = 0; pl < PL; ++pl) fb[j][pl] = sB[buf][(pl * BN + row) * 2 + (h ^ swz(row))];
    }
    // term pairs (ta, tb) with ta + tb < NT
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int s = NT - 1; s >= 0; --s)          // small terms first
#pragma unroll
          for (int ta = 0; ta <= s; ++ta) {
            const int tb = s - ta;
            accR[i][j] = mfma16<BF>(fa[i][ta], fb[j][tb], accR[i][j]);
            accR[i][j] = mfma16<BF>(na[i][ta], fb[j][NT + tb], accR[i][j]);
            accI[i][j] = mfma16<BF>(fa[i][ta], fb[j][NT + tb], accI[i][j]);
            accI[i][j] = mfma16<BF>(fa[i][NT + ta], fb[j][tb], accI[i][j]);
          }
    if (more) {
#pragma unroll
      for (int s = 0; s < NA; ++s) sA[buf ^ 1][la[s]] = ra[s];
#pragma unroll
      for (int s = 0; s < NBL; ++s) sB[buf ^ 1][lb[s]] = rb[s];
    }
    __syncthreads();
  }

  if (tail >= 0) {
    constexpr int unit = 2 * MB * NB * 16 * kThreads;
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
    __threadfence();
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(a.cnt + tail, 1) == a.split - 1;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const float *pt = a.part + (size_t)tail * a.split * unit + tid;
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        accR[i][j] = v16f{0};
        accI[i][j] = v16f{0};
      }
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
    if (tid == 0) a.cnt[tail] = 0;
  }

  // epilogue; accumulator item r of lane (l32, h): row 8 (r/4) + 4 h + r % 4, column l32
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = n0 + wn * WTN + j * 32 + l32;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int mb = m0 + wm * WTM + i * 32 + 8 * g + 4 * h;
        if (EPI == EPI_STORE) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const size_t o = (size_t)(mb + q) * a.ldc + n;
            a.cr[o] = accR[i][j][4 * g + q];
            a.ci[o] = accI[i][j][4 * g + q];
          }
        } else {
          unsigned short tr[NT][4], ti[NT][4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float cr = accR[i][j][4 * g + q], ci = accI[i][j][4 * g + q];
            const float am = a.amp[(size_t)(mb + q) * a.ldc + n];
            const float mag2 = cr * cr + ci * ci;
            float pr = 0.f, pi = 0.f;
            if (am > 0.f) {
              if (mag2 > 0.f) {
                const float sc = am * rsqrtf(mag2);
                pr = cr * sc;
                pi = ci * sc;
              } else {
                pr = am;
              }
            }
            split_terms<BF, NT>(pr, &tr[0][q], 4);
            split_terms<BF, NT>(pi, &ti[0][q], 4);
          }
#pragma unroll
          for (int s = 0; s < NT; ++s) {
            const u2 vr = {(unsigned)tr[s][0] | ((unsigned)tr[s][1] << 16),
                           (unsigned)tr[s][2] | ((unsigned)tr[s][3] << 16)};
            const u2 vi = {(unsigned)ti[s][0] | ((unsigned)ti[s][1] << 16),
                           (unsigned)ti[s][2] | ((unsigned)ti[s][3] << 16)};
            *reinterpret_cast<u2 *>(a.pt + (size_t)s * a.pt_plane + (size_t)n * a.M + mb) = vr;
            *reinterpret_cast<u2 *>(a.pt + (size_t)(NT + s) * a.pt_plane + (size_t)n * a.M + mb) =
                vi;
          }
        }
      }
    }
}

template <int BM, int BN, bool BF, int NT, int EPI>
hipError_t launch_t(const SplitArgs &args, int grid, hipStream_t s) {
  hipLaunchKernelGGL((cgemm_split_mfma<BM, BN, BF, NT, EPI>), dim3(grid), dim3(kThreads), 0, s,
                     args);
  return hipGetLastError();
}

template <bool BF, int NT, int EPI>
hipError_t launch_e(int bm, int bn, const SplitArgs &args, int grid, hipStream_t s) {
  if (bm == 64 && bn == 64) return launch_t<64, 64, BF, NT, EPI>(args, grid, s);
  if (bm == 128 && bn == 64) return launch_t<128, 64, BF, NT, EPI>(args, grid, s);
  if (bm == 64 && bn == 128) return launch_t<64, 128, BF, NT, EPI>(args, grid, s);
  if (bm == 128 && bn == 128) return launch_t<128, 128, BF, NT, EPI>(args, grid, s);
  return hipErrorInvalidValue;
}

template <int EPI>
hipError_t launch_p(int precision, int bm, int bn, const SplitArgs &args, int grid,
                    hipStream_t s) {
  switch (precision) {
    case GSWMTP_BF16X3: return launch_e<true, 2, EPI>(bm, bn, args, grid, s);
    case GSWMTP_FP16X3: return launch_e<false, 2, EPI>(bm, bn, args, grid, s);
    case GSWMTP_BF16X6: return launch_e<true, 3, EPI>(bm, bn, args, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_cgemm_split(const gswmtp_plan *p, bool forward, int epi,
                              const unsigned short *bt, float *cr, float *ci,
                              unsigned short *pt_out, bool honour_done, hipStream_t s) {
  const Dims &d = p->d;
  const GemmSched &sc = forward ? p->sched_fwd : p->sched_bwd;
  const int nt = split_terms_of(p->precision);
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
  a.cnt = p->b.tickets;
  if (nt < 2 || a.M % sc.tile.bm || a.N % sc.tile.bn || a.K % kBK) return hipErrorInvalidValue;
  if (sc.tiles_m * sc.tile.bm != a.M || sc.tiles * sc.tile.bm * sc.tile.bn != a.M * a.N)
    return hipErrorInvalidValue;
  if (epi == EPI_PROJECT && (forward || !pt_out)) return hipErrorInvalidValue;
  a.tiles_m = sc.tiles_m;
  a.t_dp = sc.t_dp;
  a.split = sc.split;
  if (epi == EPI_STORE) return launch_p<EPI_STORE>(p->precision, sc.tile.bm, sc.tile.bn, a, sc.grid, s);
  if (epi == EPI_PROJECT)
    return launch_p<EPI_PROJECT>(p->precision, sc.tile.bm, sc.tile.bn, a, sc.grid, s);
  return hipErrorInvalidValue;
}

}  // namespace gswmtp
