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
// stages of 16 complex values staged through LDS with double buffering and a
// register prefetch of the next stage.
//
// Epilogues: store C; project onto the amplitude constraint
// (E = A C / |C|, phasor 1 where C = 0: the phase-only projection of
// Algorithm 1, fused so E' never reaches HBM); or the phase-gradient
// 2 Im(conj(E) C).
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
  int lda, ldb, ldc;
  int M, N, K;
  int tiles_m, tiles;
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

template <int BM, int BN, int EPI>
__global__ __launch_bounds__(kThreads) void cgemm_f32_mfma(CgemmArgs a) {
  if (a.done && *a.done) return;
  constexpr int WTM = BM / 2, WTN = BN / 2;    // wave tile (complex)
  constexpr int MB = WTM / 32, NB = WTN / 32;  // 32x32 blocks per wave
  constexpr int SA = BM + 32, SB = BN + 32;    // padded LDS row pitch (floats)
  constexpr int A4 = kBK * BM / 4;             // float4 per A plane per stage
  constexpr int B4 = kBK * BN / 4;
  constexpr int NA = 2 * A4 / kThreads, NBL = 2 * B4 / kThreads;
  static_assert(2 * A4 % kThreads == 0 && 2 * B4 % kThreads == 0, "tile/thread mismatch");

  __shared__ float sA[2][2][kBK * SA];
  __shared__ float sB[2][2][kBK * SB];

  const int tid = threadIdx.x;
  const int t = xcd_tile(blockIdx.x, a.tiles);
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

  // Staging map: float4 s of this thread covers plane s / (NA / 2) of the
  // tile, row k = (idx % A4) / (BM / 4), columns 4 m4 .. 4 m4 + 3.
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

  const int KT = a.K / kBK;
#pragma unroll
  for (int s = 0; s < NA; ++s) ra[s] = *reinterpret_cast<const v4f *>(ga[s]);
#pragma unroll
  for (int s = 0; s < NBL; ++s) rb[s] = *reinterpret_cast<const v4f *>(gb[s]);
#pragma unroll
  for (int s = 0; s < NA; ++s) *reinterpret_cast<v4f *>(&sA[0][0][la[s]]) = ra[s];
#pragma unroll
  for (int s = 0; s < NBL; ++s) *reinterpret_cast<v4f *>(&sB[0][0][lb[s]]) = rb[s];
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < KT) {
#pragma unroll
      for (int s = 0; s < NA; ++s)
        ra[s] = *reinterpret_cast<const v4f *>(ga[s] + (size_t)(kt + 1) * stepA);
#pragma unroll
      for (int s = 0; s < NBL; ++s)
        rb[s] = *reinterpret_cast<const v4f *>(gb[s] + (size_t)(kt + 1) * stepB);
    }
    const float *pa = &sA[buf][0][0];
    const float *pb = &sB[buf][0][0];
#pragma unroll
    for (int p = 0; p < kBK / 2; ++p) {
      const int k = 2 * p + h;   // lanes 0-31 take k = 2p, lanes 32-63 k = 2p + 1
      float ar[MB], ai[MB], br[NB], bi[NB];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        ar[i] = pa[k * SA + wm * WTM + i * 32 + l32];
        ai[i] = pa[kBK * SA + k * SA + wm * WTM + i * 32 + l32];
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        br[j] = pb[k * SB + wn * WTN + j * 32 + l32];
        bi[j] = pb[kBK * SB + k * SB + wn * WTN + j * 32 + l32];
      }
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          accR[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[i], br[j], accR[i][j], 0, 0, 0);
          accR[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai[i], bi[j], accR[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[i], bi[j], accI[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[i], br[j], accI[i][j], 0, 0, 0);
        }
    }
    if (kt + 1 < KT) {
      float *qa = &sA[buf ^ 1][0][0];
      float *qb = &sB[buf ^ 1][0][0];
#pragma unroll
      for (int s = 0; s < NA; ++s) *reinterpret_cast<v4f *>(&qa[la[s]]) = ra[s];
#pragma unroll
      for (int s = 0; s < NBL; ++s) *reinterpret_cast<v4f *>(&qb[lb[s]]) = rb[s];
    }
    __syncthreads();
  }

  // Accumulator layout of the 32x32 f32 block: lane (l32, h), item r holds
  // row 8 (r / 4) + 4 h + r % 4, column l32.
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * WTM + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        const int n = n0 + wn * WTN + j * 32 + l32;
        const size_t o = (size_t)m * a.ldc + n;
        float cr = accR[i][j][r], ci = accI[i][j][r];
        if (EPI == EPI_STORE) {
          a.cr[o] = cr;
          a.ci[o] = ci;
        } else if (EPI == EPI_PROJECT) {
          const float am = a.amp[o];
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
          a.cr[o] = pr;
          a.ci[o] = pi;
        } else {
          a.cr[o] = 2.f * (a.er[o] * ci - a.ei[o] * cr);
        }
      }
}

template <int BM, int BN, int EPI>
hipError_t launch_t(const CgemmArgs &args, hipStream_t s) {
  hipLaunchKernelGGL((cgemm_f32_mfma<BM, BN, EPI>), dim3(args.tiles), dim3(kThreads), 0, s,
                     args);
  return hipGetLastError();
}

template <int EPI>
hipError_t launch_e(int bm, int bn, const CgemmArgs &args, hipStream_t s) {
  if (bm == 64 && bn == 64) return launch_t<64, 64, EPI>(args, s);
  if (bm == 64 && bn == 128) return launch_t<64, 128, EPI>(args, s);
  if (bm == 128 && bn == 64) return launch_t<128, 64, EPI>(args, s);
  if (bm == 128 && bn == 128) return launch_t<128, 128, EPI>(args, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_cgemm(const gswmtp_plan *p, bool forward, int epi, const float *br,
                        const float *bi, float *cr, float *ci, const float *er,
                        const float *ei, bool honour_done, hipStream_t s) {
  const Dims &d = p->d;
  const GemmTile &tl = forward ? p->tile_fwd : p->tile_bwd;
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
  if (a.M % tl.bm || a.N % tl.bn || a.K % kBK) return hipErrorInvalidValue;
  a.tiles_m = a.M / tl.bm;
  a.tiles = a.tiles_m * (a.N / tl.bn);
  switch (epi) {
    case EPI_STORE: return launch_e<EPI_STORE>(tl.bm, tl.bn, a, s);
    case EPI_PROJECT: return launch_e<EPI_PROJECT>(tl.bm, tl.bn, a, s);
    case EPI_GRAD: return launch_e<EPI_GRAD>(tl.bm, tl.bn, a, s);
  }
  return hipErrorInvalidValue;
}

const char *cgemm_kernel_name(const gswmtp_plan *, bool, int) { return "cgemm_f32_mfma"; }

}  // namespace gswmtp
