// Focal-plane stages of a GSW-MTP pass: the focus statistics and generalised
// weight update of Algorithm 1 (fed by the focus gather fused into the
// forward product), and the scatter of the updated focal field back onto the
// reduced focal rows (every non-focus sample of the reduced focal grid is zero
// in the inverse propagation).
#include <cmath>
#include <cstring>

#include "gswmtp_internal.h"

namespace gswmtp {
namespace {


struct Sum {
  static constexpr double identity = 0.0;
  __device__ double operator()(double a, double b) const { return a + b; }
};
struct Max {
  static constexpr double identity = -__builtin_inf();
  __device__ double operator()(double a, double b) const { return a > b ? a : b; }
};

// One step of a wave reduction on DPP lane moves (no LDS round trip): lanes
// of the rows in ROWS combine with the value CTRL moves to them, the other
// lanes with the identity.
template <int CTRL, int ROWS, typename Op>
__device__ __forceinline__ double dpp_step(double v, Op op) {
  const long long b = __double_as_longlong(v), e = __double_as_longlong(Op::identity);
  const int lo = __builtin_amdgcn_update_dpp((int)e, (int)b, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(e >> 32), (int)(b >> 32), CTRL, ROWS, 0xf,
                                             false);
  return op(v, __longlong_as_double(((long long)hi << 32) | (unsigned)lo));
}

// Deterministic reductions over one kUpdThreads workgroup: a fixed DPP
// sequence inside each wave (lane pairs, quads, half rows, rows by mirroring,
// then rows 0 + 1 and 2 + 3 and the two halves by row broadcasts; the total
// ends in lane 63), then the kUpdThreads / 64 wave results added in wave
// order by every thread (one barrier; each call site uses its own LDS slots).
template <typename Op>
__device__ __forceinline__ double wave_reduce(double v, Op op) {
  v = dpp_step<0xB1, 0xf>(v, op);    // quad_perm [1, 0, 3, 2]
  v = dpp_step<0x4E, 0xf>(v, op);    // quad_perm [2, 3, 0, 1]
  v = dpp_step<0x141, 0xf>(v, op);   // row_half_mirror
  v = dpp_step<0x140, 0xf>(v, op);   // row_mirror
  v = dpp_step<0x142, 0xa>(v, op);   // row_bcast:15 into rows 1 and 3
  v = dpp_step<0x143, 0xc>(v, op);   // row_bcast:31 into rows 2 and 3
  return v;                          // complete in lane 63
}
template <int NV, typename Op>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double (*slot)[16], Op op) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    v[q] = wave_reduce(v[q], op);
    if (lane == 63) slot[q][wave] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double r = slot[q][0];
    for (int w = 1; w < kUpdThreads / 64; ++w) r = op(r, slot[q][w]);
    v[q] = r;
  }
}


struct UpdateArgs {
  const float *gpart;      // [T][2 ldp] fused-gather partials of the forward product
  int T;                   // partials per focus
  int ldp;                 // foci per partial row (nf rounded up to even)
  float scale;             // power-of-two factor undoing the pupil scale
  float *theta;            // [2 nf] forward field (written)
  float *theta_new;        // [2 nf] updated focal field (scaled by a power of 2)
  float *intensity;        // [nf] |Theta|^2
  const double *target;    // [nf] raw target intensities
  const double *tnorm;     // [nf] target / sum(target)
  const double *tinv;      // [nf] 1 / tnorm (0 where tnorm is 0)
  const double *tsqrt;     // [nf] sqrt(target)
  double *w;               // [nf]
  double *fixph;           // [2 nf] frozen focal phasors (phase fixing)
  double *stats;           // ST_*
  double *hist;            // [3 kHistCap]
  int *ctrl;               // CTRL_*
  double *s1, *s2;         // many-focus form: per-workgroup partial sums [nwg], [5 nwg]
  int *snap;               // many-focus form: control values at the start of the pass
  int nwg;                 // many-focus form: workgroups (ceil(nf / kUpdThreads))
  int nf;
  int mode;                // UPD_ITERATE or UPD_STATS
  int weighting;           // GSWMTP_WEIGHT_*
  double n_ap, sum_a2;
  const double *meas;      // [nf] measured intensities at unit sum (camera in the loop):
                           // the weight update's i, in place of |Theta|^2 / sum; or null
};

// Unit phasor Theta / |Theta| (1 at a dark focus) from float64 parts: one
// reciprocal square root, accurate far beyond the float32 field it scales.
__device__ __forceinline__ void unit_phasor(double re, double im, double &pr, double &pi) {
  const double m2 = re * re + im * im;
  pr = 1.0;
  pi = 0.0;
  if (m2 > 0.0) {
    const double r = __builtin_amdgcn_rsq(m2);
    pr = re * r;
    pi = im * r;
  }
}

// Algorithm 1 between the two propagations, for all foci, in one workgroup:
//   Theta_n = sum of the forward product's gather partials (fixed order);
//   I_n = |Theta_n|^2; accuracy xi from unit-sum intensities; efficiency and
//   uniformity; termination test (before any update); weight update
//   w <- w sqrt(t / max(i, 1e-30)); new focal field w sqrt(target) Theta/|Theta|
//   (phasor 1 at a dark focus), written scaled by 2^e so its largest
//   magnitude is in [0.5, 1) - the phase projection discards the scale.
// All reductions are float64 in a fixed order.
// Sums and maxima of several values in one pass: one barrier for all.
template <int NS, int NM>
__device__ __forceinline__ void block_reduce_mixed(double (&sv)[NS], double (&mv)[NM],
                                                   double (*slot)[16]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    sv[q] = wave_reduce(sv[q], Sum());
    if (lane == 63) slot[q][wave] = sv[q];
  }
#pragma unroll
  for (int q = 0; q < NM; ++q) {
    mv[q] = wave_reduce(mv[q], Max());
    if (lane == 63) slot[NS + q][wave] = mv[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    double r = slot[q][0];
    for (int w = 1; w < kUpdThreads / 64; ++w) r += slot[q][w];
    sv[q] = r;
  }
#pragma unroll
  for (int q = 0; q < NM; ++q) {
    double r = slot[NS + q][0];
    for (int w = 1; w < kUpdThreads / 64; ++w) r = r > slot[NS + q][w] ? r : slot[NS + q][w];
    mv[q] = r;
  }
}

// Per-focus values live in registers (FPT consecutive foci per thread,
// n = FPT t + f, so one 16-byte load reads a partial of a pair of foci).
// Two reductions: sum I first; then, from it, the accuracy and uniformity
// terms and the new weights' amplitude maximum together (everything needed
// for the termination test and the update), so only one more barrier.  The
// partials are read in predicated chunks of 16 loads, all in flight at once.
template <int FPT>
__device__ __forceinline__ void focus_update_body(const UpdateArgs &a, double (*slots)[16]) {
  const int t = threadIdx.x;
  const bool upd = a.mode == UPD_ITERATE;
  // every small control value is read up front, beside the per-focus data,
  // so no load latency is left on the path after the reductions
  const double X = upd ? a.stats[ST_STOP] : 0.0;
  const int hist0 = upd && t == 0 ? a.ctrl[CTRL_HIST] : 0;
  const int iters0 = upd ? a.ctrl[CTRL_ITERS] : 0;
  // phase fixing (Sec. 2): from updating pass fix_k on, the focal phasors
  // are the ones recorded by the first such pass
  const int fix_k = upd ? a.ctrl[CTRL_FIX] : 0;
  const bool fixing = fix_k > 0 && iters0 + 1 >= fix_k;
  const bool recorded = fixing && a.ctrl[CTRL_FIXED] != 0;
  double tn[FPT], tiv[FPT], tg[FPT], wv[FPT], fpr[FPT], fpi[FPT], mi[FPT];
  float thr[FPT], thi[FPT];
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    const int n = FPT * t + f;
    const bool ok = n < a.nf;
    mi[f] = ok && upd && a.meas ? a.meas[n] : 0.0;
    tn[f] = ok ? a.tnorm[n] : 0.0;
    tiv[f] = ok ? a.tinv[n] : 0.0;
    tg[f] = ok && upd ? a.tsqrt[n] : 0.0;
    wv[f] = ok && upd ? a.w[n] : 0.0;
    fpr[f] = ok && recorded ? a.fixph[2 * n] : 1.0;
    fpi[f] = ok && recorded ? a.fixph[2 * n + 1] : 0.0;
  }
  static_assert(FPT == 2, "one 16-byte partial load per pair of foci");
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int CHUNK = 16;
#pragma unroll
  for (int f = 0; f < FPT; ++f) thr[f] = thi[f] = 0.f;
  // partials in ascending order; one chunk in flight.  Row q holds the pair
  // (2t, 2t + 1) in 16 bytes (rows of ldp foci, ldp even); the second focus
  // of the last pair is padding when nf is odd, and ignored.
  const bool pair_on = 2 * t < a.nf;
  for (int q = 0; q < a.T; q += CHUNK) {
    f4 v[CHUNK];
#pragma unroll
    for (int j = 0; j < CHUNK; ++j)
      v[j] = q + j < a.T && pair_on
                 ? *reinterpret_cast<const f4 *>(a.gpart + 2 * ((size_t)(q + j) * a.ldp + 2 * t))
                 : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < CHUNK; ++j) {   // zeros past T: exact no-ops
      thr[0] += v[j].x;
      thi[0] += v[j].y;
      thr[1] += v[j].z;
      thi[1] += v[j].w;
    }
  }
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    thr[f] *= a.scale;
    thi[f] *= a.scale;
  }
  if (upd && a.ctrl[CTRL_DONE]) return;   // read while the partials were in flight
  double v1[1] = {0.0};
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    const int n = FPT * t + f;
    if (n >= a.nf) continue;
    a.theta[2 * n] = thr[f];
    a.theta[2 * n + 1] = thi[f];
    const double I = (double)thr[f] * thr[f] + (double)thi[f] * thi[f];
    a.intensity[n] = (float)I;
    v1[0] += I;
  }
  block_reduce<1>(v1, &slots[0], Sum());
  const double sI = v1[0];
  const double inv = sI > 0.0 ? 1.0 / sI : 0.0;

  // accuracy / uniformity terms and the new weights (not yet written)
  double sv[2] = {0.0, 0.0};                       // sum (t - i)^2, sum i^2
  double mv[3] = {-INFINITY, -INFINITY, 0.0};      // max r, max -r, max new amplitude
  double amag[FPT];
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    amag[f] = 0.0;
    if (FPT * t + f >= a.nf) continue;
    const double re = thr[f], im = thi[f];
    const double in = (re * re + im * im) * inv;
    sv[0] += (tn[f] - in) * (tn[f] - in);
    sv[1] += in * in;
    if (tn[f] > 0.0) {
      const double r = in * tiv[f];
      mv[0] = r > mv[0] ? r : mv[0];
      mv[1] = -r > mv[1] ? -r : mv[1];
    }
    if (upd) {
      const double iw = a.meas ? mi[f] : in;
      if (a.weighting == GSWMTP_WEIGHT_GSW) wv[f] *= sqrt(tn[f] / (iw > 1e-30 ? iw : 1e-30));
      amag[f] = wv[f] * tg[f];
      mv[2] = amag[f] > mv[2] ? amag[f] : mv[2];
    }
  }
  block_reduce_mixed<2, 3>(sv, mv, &slots[1]);
  const double d2 = sv[0], i2 = sv[1], rmax = mv[0], rmin = -mv[1], amax = mv[2];

  const double xi = i2 > 0.0 ? 1.0 - sqrt(d2) / sqrt(i2) : -INFINITY;
  const double eta = sI / (a.n_ap * a.sum_a2);
  const double U = (rmax + rmin) > 0.0 ? 1.0 - (rmax - rmin) / (rmax + rmin) : 0.0;
  int stop = 0;
  if (upd) {
    if (!isfinite(sI)) stop = 1;
    if (X > 0.0 && xi > X) stop = 1;
  }
  if (t == 0) {
    a.stats[ST_XI] = xi;
    a.stats[ST_ETA] = eta;
    a.stats[ST_U] = U;
    a.stats[ST_SUMI] = sI;
    if (upd) {
      double *e = a.hist + 3 * (hist0 % kHistCap);
      e[0] = xi;
      e[1] = eta;
      e[2] = U;
      a.ctrl[CTRL_HIST] = hist0 + 1;
      if (!isfinite(sI)) a.ctrl[CTRL_NONFINITE] = 1;
      if (stop) a.ctrl[CTRL_DONE] = 1;
    }
  }
  if (!upd || stop) return;

  // weights and the new focal field, scaled by 2^e (max magnitude in [0.5, 1))
  int e = 0;
  if (amax > 0.0 && isfinite(amax)) e = -ilogb(amax) - 1;
  const double scale = ldexp(1.0, e);
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    const int n = FPT * t + f;
    if (n >= a.nf) continue;
    if (a.weighting == GSWMTP_WEIGHT_GSW) a.w[n] = wv[f];
    double pr = 1.0, pi = 0.0;
    if (recorded) {
      pr = fpr[f];
      pi = fpi[f];
    } else {
      unit_phasor(thr[f], thi[f], pr, pi);
      if (fixing) {
        a.fixph[2 * n] = pr;
        a.fixph[2 * n + 1] = pi;
      }
    }
    const double am = amag[f] * scale;
    a.theta_new[2 * n] = (float)(am * pr);
    a.theta_new[2 * n + 1] = (float)(am * pi);
  }
  if (t == 0) {
    a.ctrl[CTRL_ITERS] = iters0 + 1;
    if (fixing && !recorded) a.ctrl[CTRL_FIXED] = 1;
  }
}

// Many foci (more than one workgroup holds in registers): the same update in
// three launches over nwg = ceil(nf / kUpdThreads) workgroups, one focus per
// thread, with no synchronisation between workgroups.  Phase 1 forms Theta,
// I and per-workgroup sums of I; phase 2 reduces those sums (every workgroup
// alike, fixed order), forms the accuracy / uniformity terms and the new
// amplitudes, and writes their per-workgroup sums and maxima; phase 3
// reduces those, takes the termination test and writes the weights and the
// new focal field.  Control values are read by phase 1 into a snapshot, so
// phase 3's writes to the control block cannot race with its own reads.
enum { SNAP_DONE = 0, SNAP_ITERS = 1, SNAP_FIX = 2, SNAP_FIXED = 3, SNAP_HIST = 4 };

__device__ __forceinline__ void big_phase1(const UpdateArgs &a, int b, double (*slots)[16]) {
  const int t = threadIdx.x, n = b * kUpdThreads + t;
  const bool upd = a.mode == UPD_ITERATE;
  if (b == 0 && t == 0) {
    a.snap[SNAP_DONE] = upd ? a.ctrl[CTRL_DONE] : 0;
    a.snap[SNAP_ITERS] = a.ctrl[CTRL_ITERS];
    a.snap[SNAP_FIX] = a.ctrl[CTRL_FIX];
    a.snap[SNAP_FIXED] = a.ctrl[CTRL_FIXED];
    a.snap[SNAP_HIST] = a.ctrl[CTRL_HIST];
  }
  typedef float f2 __attribute__((ext_vector_type(2)));
  const f2 *gp = reinterpret_cast<const f2 *>(a.gpart);
  constexpr int CHUNK = 32;
  float sr = 0.f, si = 0.f;
  for (int q = 0; q < a.T; q += CHUNK) {
    f2 v[CHUNK];
#pragma unroll
    for (int j = 0; j < CHUNK; ++j)
      v[j] = q + j < a.T && n < a.nf ? gp[(size_t)(q + j) * a.ldp + n] : f2{0.f, 0.f};
#pragma unroll
    for (int j = 0; j < CHUNK; ++j) {   // zeros past T: exact no-ops
      sr += v[j].x;
      si += v[j].y;
    }
  }
  sr *= a.scale;
  si *= a.scale;
  if (upd && a.ctrl[CTRL_DONE]) return;
  double v1[1] = {0.0};
  if (n < a.nf) {
    a.theta[2 * n] = sr;
    a.theta[2 * n + 1] = si;
    const double I = (double)sr * sr + (double)si * si;
    a.intensity[n] = (float)I;
    v1[0] = I;
  }
  block_reduce<1>(v1, &slots[0], Sum());
  if (t == 0) a.s1[b] = v1[0];
}

// Sum of the phase-1 partials, identical in every workgroup.
__device__ __forceinline__ double big_sum_I(const UpdateArgs &a, double (*slots)[16]) {
  double v[1] = {0.0};
  for (int j = threadIdx.x; j < a.nwg; j += kUpdThreads) v[0] += a.s1[j];
  block_reduce<1>(v, &slots[0], Sum());
  return v[0];
}

// Per-focus terms of phase 2 / phase 3 (the same arithmetic in both).
struct BigFocus {
  double in, tn, w_new, amag;
  float re, im;
};
__device__ __forceinline__ BigFocus big_focus(const UpdateArgs &a, int n, double inv, bool upd) {
  BigFocus f{};
  f.re = a.theta[2 * n];
  f.im = a.theta[2 * n + 1];
  const double re = f.re, im = f.im;
  f.in = (re * re + im * im) * inv;
  f.tn = a.tnorm[n];
  if (upd) {
    double w = a.w[n];
    const double iw = a.meas ? a.meas[n] : f.in;
    if (a.weighting == GSWMTP_WEIGHT_GSW) w *= sqrt(f.tn / (iw > 1e-30 ? iw : 1e-30));
    f.w_new = w;
    f.amag = w * a.tsqrt[n];
  }
  return f;
}

__device__ __forceinline__ void big_phase2(const UpdateArgs &a, int b, double (*slots)[16]) {
  const bool upd = a.mode == UPD_ITERATE;
  if (upd && a.snap[SNAP_DONE]) return;
  const int t = threadIdx.x, n = b * kUpdThreads + t;
  const double sI = big_sum_I(a, slots);
  const double inv = sI > 0.0 ? 1.0 / sI : 0.0;
  double sv[2] = {0.0, 0.0}, mv[3] = {-INFINITY, -INFINITY, 0.0};
  if (n < a.nf) {
    const BigFocus f = big_focus(a, n, inv, upd);
    sv[0] = (f.tn - f.in) * (f.tn - f.in);
    sv[1] = f.in * f.in;
    if (f.tn > 0.0) {
      const double r = f.in * a.tinv[n];
      mv[0] = r;
      mv[1] = -r;
    }
    if (upd) mv[2] = f.amag;
  }
  block_reduce_mixed<2, 3>(sv, mv, &slots[1]);
  if (t == 0) {
    a.s2[5 * b] = sv[0];
    a.s2[5 * b + 1] = sv[1];
    a.s2[5 * b + 2] = mv[0];
    a.s2[5 * b + 3] = mv[1];
    a.s2[5 * b + 4] = mv[2];
  }
}

__device__ __forceinline__ void big_phase3(const UpdateArgs &a, int b, double (*slots)[16]) {
  const bool upd = a.mode == UPD_ITERATE;
  if (upd && a.snap[SNAP_DONE]) return;
  const int t = threadIdx.x, n = b * kUpdThreads + t;
  const double sI = big_sum_I(a, slots);
  const double inv = sI > 0.0 ? 1.0 / sI : 0.0;
  double sv[2] = {0.0, 0.0}, mv[3] = {-INFINITY, -INFINITY, 0.0};
  for (int j = t; j < a.nwg; j += kUpdThreads) {
    sv[0] += a.s2[5 * j];
    sv[1] += a.s2[5 * j + 1];
    mv[0] = a.s2[5 * j + 2] > mv[0] ? a.s2[5 * j + 2] : mv[0];
    mv[1] = a.s2[5 * j + 3] > mv[1] ? a.s2[5 * j + 3] : mv[1];
    mv[2] = a.s2[5 * j + 4] > mv[2] ? a.s2[5 * j + 4] : mv[2];
  }
  block_reduce_mixed<2, 3>(sv, mv, &slots[1]);
  const double d2 = sv[0], i2 = sv[1], rmax = mv[0], rmin = -mv[1], amax = mv[2];
  const double xi = i2 > 0.0 ? 1.0 - sqrt(d2) / sqrt(i2) : -INFINITY;
  const double eta = sI / (a.n_ap * a.sum_a2);
  const double U = (rmax + rmin) > 0.0 ? 1.0 - (rmax - rmin) / (rmax + rmin) : 0.0;
  int stop = 0;
  if (upd) {
    if (!isfinite(sI)) stop = 1;
    const double X = a.stats[ST_STOP];
    if (X > 0.0 && xi > X) stop = 1;
  }
  if (b == 0 && t == 0) {
    a.stats[ST_XI] = xi;
    a.stats[ST_ETA] = eta;
    a.stats[ST_U] = U;
    a.stats[ST_SUMI] = sI;
    if (upd) {
      const int h = a.snap[SNAP_HIST];
      double *e = a.hist + 3 * (h % kHistCap);
      e[0] = xi;
      e[1] = eta;
      e[2] = U;
      a.ctrl[CTRL_HIST] = h + 1;
      if (!isfinite(sI)) a.ctrl[CTRL_NONFINITE] = 1;
      if (stop) a.ctrl[CTRL_DONE] = 1;
    }
  }
  if (!upd || stop) return;
  int e = 0;
  if (amax > 0.0 && isfinite(amax)) e = -ilogb(amax) - 1;
  const double scale = ldexp(1.0, e);
  const int iters0 = a.snap[SNAP_ITERS], fix_k = a.snap[SNAP_FIX];
  const bool fixing = fix_k > 0 && iters0 + 1 >= fix_k;
  const bool recorded = fixing && a.snap[SNAP_FIXED] != 0;
  if (n < a.nf) {
    const BigFocus f = big_focus(a, n, inv, true);
    if (a.weighting == GSWMTP_WEIGHT_GSW) a.w[n] = f.w_new;
    double pr = 1.0, pi = 0.0;
    if (recorded) {
      pr = a.fixph[2 * n];
      pi = a.fixph[2 * n + 1];
    } else {
      unit_phasor(f.re, f.im, pr, pi);
      if (fixing) {
        a.fixph[2 * n] = pr;
        a.fixph[2 * n + 1] = pi;
      }
    }
    const double am = f.amag * scale;
    a.theta_new[2 * n] = (float)(am * pr);
    a.theta_new[2 * n + 1] = (float)(am * pi);
  }
  if (b == 0 && t == 0) {
    a.ctrl[CTRL_ITERS] = iters0 + 1;
    if (fixing && !recorded) a.ctrl[CTRL_FIXED] = 1;
  }
}

constexpr int kUpdRegFoci = kUpdRegFociMax / kUpdThreads;   // foci per thread in registers

__global__ __launch_bounds__(kUpdThreads) void focus_update(UpdateArgs a) {
  __shared__ double slots[8][16];
  focus_update_body<kUpdRegFoci>(a, slots);
}

template <int PHASE>
__global__ __launch_bounds__(kUpdThreads) void focus_update_big(UpdateArgs a) {
  __shared__ double slots[8][16];
  if constexpr (PHASE == 1) big_phase1(a, blockIdx.x, slots);
  else if constexpr (PHASE == 2) big_phase2(a, blockIdx.x, slots);
  else big_phase3(a, blockIdx.x, slots);
}

// Grouped over the plans of a batch.  Phase 1 launch: item h owns blocks
// [starts[h], starts[h+1]); a plan in the register form (nwg == 0 in its
// arguments) has one block that runs its whole update; a many-focus plan
// runs phase 1 on nwg blocks.  Phases 2 and 3 run over the many-focus plans
// only (their own item table).
template <int PHASE>
__global__ __launch_bounds__(kUpdThreads) void focus_update_grouped(const UpdateArgs *items,
                                                                    const int *starts, int n) {
  __shared__ double slots[8][16];
  const int bid = blockIdx.x;
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (starts[mid] <= bid) lo = mid; else hi = mid;
  }
  const UpdateArgs a = items[lo];
  const int b = bid - starts[lo];
  if constexpr (PHASE == 1) {
    if (a.nwg == 0) focus_update_body<kUpdRegFoci>(a, slots);
    else big_phase1(a, b, slots);
  } else if constexpr (PHASE == 2) {
    big_phase2(a, b, slots);
  } else {
    big_phase3(a, b, slots);
  }
}

// Grid form of the focus gather: Theta_n is entry (ir_n, ic_n) of the dense
// reduced grid G (written as the single gather partial of focus n).
__global__ void grid_gather(const float *__restrict__ gr, const float *__restrict__ gi, int ldg,
                            const int *__restrict__ ir, const int *__restrict__ ic, int nf,
                            float *__restrict__ gpart) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nf) return;
  const size_t o = (size_t)ir[n] * ldg + ic[n];
  gpart[2 * n] = gr[o];
  gpart[2 * n + 1] = gi[o];
}

// Grid form of the scatter: Theta'_n onto the transposed grid at (ic_n, ir_n);
// every other entry of the grid stays zero from plan creation.  With g (the
// phase gradient's focal weights) the value placed is g_n Theta_n, the same
// product grad_field forms.
__global__ void grid_scatter(const float *__restrict__ tn, float scale, const int *__restrict__ ir,
                             const int *__restrict__ ic, int nf, float *__restrict__ tr,
                             float *__restrict__ ti, int ldt, const float *__restrict__ g) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nf) return;
  const size_t o = (size_t)ic[n] * ldt + ir[n];
  float a = tn[2 * n], b = tn[2 * n + 1];
  if (g) {
    a = g[n] * a;
    b = g[n] * b;
  }
  tr[o] = a * scale;
  ti[o] = b * scale;
}

// Grid form of the focus field: Theta_n = G[ir_n][ic_n] (scaled) and I_n,
// the values grid_gather and gather_reduce give (one partial from zero).
__global__ void grid_field(const float *__restrict__ gr, const float *__restrict__ gi, int ldg,
                           const int *__restrict__ ir, const int *__restrict__ ic, int nf,
                           float scale, float *__restrict__ theta, float *__restrict__ intensity,
                           float *__restrict__ theta2, float *__restrict__ intensity2) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nf) return;
  const size_t o = (size_t)ir[n] * ldg + ic[n];
  float sr = 0.f, si = 0.f;
  sr += gr[o];
  si += gi[o];
  sr *= scale;
  si *= scale;
  theta[2 * n] = sr;
  theta[2 * n + 1] = si;
  if (theta2) {
    theta2[2 * n] = sr;
    theta2[2 * n + 1] = si;
  }
  const float I = (float)((double)sr * sr + (double)si * si);
  intensity[n] = I;
  if (intensity2) intensity2[n] = I;
}

// Theta_n from the gather partials alone (operator-level forward calls, and
// the field of the current phase when no statistics are asked for), and
// optionally I_n = |Theta_n|^2; theta2 / intensity2 (optional) take second
// copies.  The partials are added in ascending order and scaled as the focus
// update does, so both give the same values.
__global__ void gather_reduce(const float *__restrict__ gpart, int T, int nf, int ldp,
                              float scale, float *__restrict__ theta,
                              float *__restrict__ intensity, float *__restrict__ theta2,
                              float *__restrict__ intensity2) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nf) return;
  float sr = 0.f, si = 0.f;
#pragma unroll 8
  for (int q = 0; q < T; ++q) {
    sr += gpart[2 * ((size_t)q * ldp + n)];
    si += gpart[2 * ((size_t)q * ldp + n) + 1];
  }
  sr *= scale;
  si *= scale;
  theta[2 * n] = sr;
  theta[2 * n + 1] = si;
  if (theta2) {
    theta2[2 * n] = sr;
    theta2[2 * n + 1] = si;
  }
  if (intensity || intensity2) {
    const float I = (float)((double)sr * sr + (double)si * si);
    if (intensity) intensity[n] = I;
    if (intensity2) intensity2[n] = I;
  }
}

// Focal values for the phase gradient: g_n Theta_n.
__global__ void grad_field(const float *__restrict__ theta, const float *__restrict__ g,
                           float *__restrict__ out, int nf) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nf) return;
  out[2 * n] = g[n] * theta[2 * n];
  out[2 * n + 1] = g[n] * theta[2 * n + 1];
}

// S[a][i] = sum_{n in row a} Theta'_n conj(Wc[ic_n][i]) for all a < Urp and
// i < Cp (rows past Ur and padded columns come out zero).  Foci of a row are
// summed in ascending (ic, n) order.
struct ScatterArgs {
  const float *tn;
  const float *wr, *wi;
  const int *ic, *ptr, *foci;     // column index in CSR order; CSR row pointers; foci
  float *sr, *si;
  int Ur, Cp;
  const int *done;
};

// Row a, columns i .. i + 3 (i a multiple of 4; Cp is a multiple of 64):
// 16-byte reads of Wc and 16-byte stores of S.
__device__ __forceinline__ void focus_scatter_body(const ScatterArgs &s_, int a, int i) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const float *__restrict__ tn = s_.tn;
  const float *__restrict__ wr = s_.wr;
  const float *__restrict__ wi = s_.wi;
  const int *__restrict__ ic = s_.ic;
  const int *__restrict__ ptr = s_.ptr;
  const int *__restrict__ foci = s_.foci;
  float *__restrict__ sr = s_.sr;
  float *__restrict__ si = s_.si;
  const int Ur = s_.Ur, Cp = s_.Cp;
  if (i >= Cp) return;
  f4 accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
  if (a < Ur) {
    const int p0 = ptr[a], p1 = ptr[a + 1];
    for (int p = p0; p < p1; ++p) {
      const int n = foci[p];
      const float xr = tn[2 * n], xi = tn[2 * n + 1];
      const size_t o = (size_t)ic[p] * Cp + i;   // ic in CSR order
      const f4 yr = *reinterpret_cast<const f4 *>(wr + o);
      const f4 yi = -*reinterpret_cast<const f4 *>(wi + o);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        accr[e] = fmaf(xr, yr[e], fmaf(-xi, yi[e], accr[e]));
        acci[e] = fmaf(xr, yi[e], fmaf(xi, yr[e], acci[e]));
      }
    }
  }
  if (s_.done && *s_.done) return;   // read after the sums' loads were issued
  *reinterpret_cast<f4 *>(sr + (size_t)a * Cp + i) = accr;
  *reinterpret_cast<f4 *>(si + (size_t)a * Cp + i) = acci;
}

__global__ __launch_bounds__(256) void focus_scatter(ScatterArgs a) {
  focus_scatter_body(a, blockIdx.y, 4 * (blockIdx.x * blockDim.x + threadIdx.x));
}

// Grouped over the plans of a batch: item h owns blocks [starts[h], starts[h+1]),
// (Cp / 1024) column blocks per reduced row.
__global__ __launch_bounds__(256) void focus_scatter_grouped(const ScatterArgs *items,
                                                             const int *starts, int n) {
  const int b = blockIdx.x;
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (starts[mid] <= b) lo = mid; else hi = mid;
  }
  const ScatterArgs a = items[lo];
  const int lb = b - starts[lo], bx = (a.Cp + 1023) / 1024;
  focus_scatter_body(a, lb / bx, 4 * ((lb % bx) * 256 + threadIdx.x));
}

// Split-precision scatter: the same S, written transposed as 16-bit term
// planes S^T [re/im][term][Cp][Urp] (the k-contiguous B operand of the
// split adjoint product).  A block computes a 32 (a) x 64 (i) tile of S with
// coalesced 16-byte reads of Wc (four columns of two rows per thread),
// transposes it through LDS and writes 8 consecutive a per thread and plane
// (16 bytes).  A thread's rows advance together (entry k of both rows at
// once), so their loads are in flight together.
// ic: reduced-grid column of the focus at each CSR position.
template <bool BF, int NT>
__device__ __forceinline__ void focus_scatter_split_body(
    const float *__restrict__ tn, const float *__restrict__ wr, const float *__restrict__ wi,
    const int *__restrict__ ic, const int *__restrict__ ptr, const int *__restrict__ foci,
    unsigned short *__restrict__ st, int Ur, int Urp, int Cp, float scale, const int *done,
    int bx, int by, float (*tr)[65], float (*ti)[65]) {
  const int i0 = bx * 64, a0 = by * 32;
  const int tid = threadIdx.x;
  // four consecutive columns i0 + 4 c4 .. + 3 (16-byte loads of Wc), two
  // rows a0 + rg + 16 q; a wave covers 64 columns of four rows
  const int c4 = tid & 15, rg = tid >> 4;
  constexpr int R = 2;
  typedef float f4 __attribute__((ext_vector_type(4)));
  int p0[R], len[R], kmax = 0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int a = a0 + rg + 16 * q;
    const int lo = a < Ur ? ptr[a] : 0, hi = a < Ur ? ptr[a + 1] : 0;
    p0[q] = lo;
    len[q] = hi - lo;
    kmax = len[q] > kmax ? len[q] : kmax;
  }
  f4 accr[R], acci[R];
#pragma unroll
  for (int q = 0; q < R; ++q) accr[q] = acci[q] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < kmax; ++k) {
    int n[R], c[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const bool on = k < len[q];
      n[q] = on ? foci[p0[q] + k] : 0;
      c[q] = on ? ic[p0[q] + k] : 0;
    }
    float xr[R], xi[R];
    f4 yr[R], yi[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const bool on = k < len[q];
      const size_t o = (size_t)c[q] * Cp + i0 + 4 * c4;
      xr[q] = on ? tn[2 * n[q]] * scale : 0.f;
      xi[q] = on ? tn[2 * n[q] + 1] * scale : 0.f;
      yr[q] = on ? *reinterpret_cast<const f4 *>(wr + o) : f4{0.f, 0.f, 0.f, 0.f};
      yi[q] = on ? -*reinterpret_cast<const f4 *>(wi + o) : f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (k < len[q])
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          accr[q][e] = fmaf(xr[q], yr[q][e], fmaf(-xi[q], yi[q][e], accr[q][e]));
          acci[q][e] = fmaf(xr[q], yi[q][e], fmaf(xi[q], yr[q][e], acci[q][e]));
        }
  }
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      tr[rg + 16 * q][4 * c4 + e] = accr[q][e];
      ti[rg + 16 * q][4 * c4 + e] = acci[q][e];
    }
  if (done && *done) return;   // uniform; read after the sums' loads were issued
  __syncthreads();
  const int i = tid >> 2, part = tid & 3;   // 64 columns x 4 runs of 8 a
  unsigned short vr[NT][8], vi[NT][8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    split_terms<BF, NT>(tr[8 * part + q][i], &vr[0][q], 8);
    split_terms<BF, NT>(ti[8 * part + q][i], &vi[0][q], 8);
  }
  const size_t plane = (size_t)Cp * Urp;
  const size_t off = kblk_index(i0 + i, a0 + 8 * part, Cp);   // 8 a in one k-block
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    u4 wv, wiv;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      wv[e] = (unsigned)vr[q][2 * e] | ((unsigned)vr[q][2 * e + 1] << 16);
      wiv[e] = (unsigned)vi[q][2 * e] | ((unsigned)vi[q][2 * e + 1] << 16);
    }
    *reinterpret_cast<u4 *>(st + (size_t)q * plane + off) = wv;
    *reinterpret_cast<u4 *>(st + (size_t)(NT + q) * plane + off) = wiv;
  }
}

template <bool BF, int NT>
__global__ __launch_bounds__(256) void focus_scatter_split(
    const float *__restrict__ tn, const float *__restrict__ wr, const float *__restrict__ wi,
    const int *__restrict__ ic, const int *__restrict__ ptr, const int *__restrict__ foci,
    unsigned short *__restrict__ st, int Ur, int Urp, int Cp, float scale, const int *done) {
  __shared__ float tr[32][65], ti[32][65];
  focus_scatter_split_body<BF, NT>(tn, wr, wi, ic, ptr, foci, st, Ur, Urp, Cp, scale, done,
                                   blockIdx.x, blockIdx.y, tr, ti);
}

// Left operand of the re-associated adjoint, for plans in which every
// reduced row a holds exactly one focus (its CSR position is then a): column
// a of Omega_r^H times that focus's new value, A_s = Omega_r^H diag(Theta'),
// as split planes in the layout of Omega_r^H's (k-blocked, K = reduced row).
// Then E' = Omega_r^H S = A_s B with B the conjugated Omega_c rows of the
// foci, fixed at plan time: the same sum as with the scatter's S, grouped
// the other way.  Four consecutive k of one row per thread.
template <bool BF, int NT>
__device__ __forceinline__ void scale_adjoint_body(
    const float *__restrict__ obr, const float *__restrict__ obi, const float *__restrict__ tn,
    const int *__restrict__ foci, int Ur, int Rp, int Urp, unsigned short *__restrict__ as,
    const int *done, size_t quad) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const size_t plane = (size_t)Rp * Urp;
  const size_t idx = 4 * quad;
  if (idx >= plane) return;
  // kblk_index(j, a, Rp) = (a / kKB) Rp kKB + j kKB + a % kKB
  const int a0 = (int)(idx / ((size_t)Rp * kKB)) * kKB + (int)(idx % kKB);
  const f4 vr = *reinterpret_cast<const f4 *>(obr + idx);
  const f4 vi = *reinterpret_cast<const f4 *>(obi + idx);
  float xr[4], xi[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = a0 + q;
    const int n = a < Ur ? foci[a] : 0;
    xr[q] = a < Ur ? tn[2 * n] : 0.f;
    xi[q] = a < Ur ? tn[2 * n + 1] : 0.f;
  }
  if (done && *done) return;   // read after the loads were issued
  unsigned short tr[NT][4], ti[NT][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float pr = fmaf(vr[q], xr[q], -vi[q] * xi[q]);
    const float pi = fmaf(vr[q], xi[q], vi[q] * xr[q]);
    split_terms<BF, NT>(pr, &tr[0][q], 4);
    split_terms<BF, NT>(pi, &ti[0][q], 4);
  }
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int s = 0; s < NT; ++s) {
    const u2 wr = {(unsigned)tr[s][0] | ((unsigned)tr[s][1] << 16),
                   (unsigned)tr[s][2] | ((unsigned)tr[s][3] << 16)};
    const u2 wi = {(unsigned)ti[s][0] | ((unsigned)ti[s][1] << 16),
                   (unsigned)ti[s][2] | ((unsigned)ti[s][3] << 16)};
    *reinterpret_cast<u2 *>(as + (size_t)s * plane + idx) = wr;
    *reinterpret_cast<u2 *>(as + (size_t)(NT + s) * plane + idx) = wi;
  }
}

template <bool BF, int NT>
__global__ __launch_bounds__(256) void k_scale_adjoint_split(
    const float *__restrict__ obr, const float *__restrict__ obi, const float *__restrict__ tn,
    const int *__restrict__ foci, int Ur, int Rp, int Urp, unsigned short *__restrict__ as,
    const int *done) {
  scale_adjoint_body<BF, NT>(obr, obi, tn, foci, Ur, Rp, Urp, as, done,
                             (size_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// One plan's scatter as an item of the batched form's grouped launch.
// Plans with the re-associated adjoint (scaled != 0) form Omega_r^H diag
// Theta' instead (obr, obi, as, Rp), one quad of k per thread.
struct ScatterSplitArgs {
  const float *tn, *wr, *wi;
  const int *ic, *ptr, *foci;
  unsigned short *st;
  int Ur, Urp, Cp;
  float scale;
  const int *done;
  const float *obr, *obi;
  unsigned short *as;
  int Rp, scaled;
};

template <bool BF, int NT>
__global__ __launch_bounds__(256) void focus_scatter_split_grouped(const ScatterSplitArgs *items,
                                                                   const int *starts, int n) {
  __shared__ float tr[32][65], ti[32][65];
  const int b = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (starts[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const ScatterSplitArgs &a = items[lo];
  const int u = b - starts[lo], gx = a.Cp / 64;
  if (a.scaled) {   // uniform per block
    scale_adjoint_body<BF, NT>(a.obr, a.obi, a.tn, a.foci, a.Ur, a.Rp, a.Urp, a.as, a.done,
                               (size_t)u * 256 + threadIdx.x);
    return;
  }
  focus_scatter_split_body<BF, NT>(a.tn, a.wr, a.wi, a.ic, a.ptr, a.foci, a.st, a.Ur, a.Urp,
                                   a.Cp, a.scale, a.done, u % gx, u / gx, tr, ti);
}

}  // namespace

hipError_t launch_scatter_split(const gswmtp_plan *p, const float *theta_new, float scale,
                                bool honour_done, hipStream_t s, unsigned short *out) {
  const Dims &d = p->d;
  const int *ic = p->b.csr_ic;
  unsigned short *st = out ? out : p->b.ss;
  const dim3 grid(d.Cp / 64, d.Urp / 32);
  const int *done = honour_done ? p->b.ctrl + CTRL_DONE : nullptr;
#define SCATTER_SPLIT(BF, NT)                                                                  \
  hipLaunchKernelGGL((focus_scatter_split<BF, NT>), grid, dim3(256), 0, s, theta_new, p->b.wc_r, \
                     p->b.wc_i, ic, p->b.csr_ptr, p->b.csr_foci, st, d.Ur, d.Urp, d.Cp, scale,   \
                     done)
  switch (p->precision) {
    case GSWMTP_BF16X3: SCATTER_SPLIT(true, 2); break;
    case GSWMTP_FP16X3: SCATTER_SPLIT(false, 2); break;
    case GSWMTP_BF16X6: SCATTER_SPLIT(true, 3); break;
    default: return hipErrorInvalidValue;
  }
#undef SCATTER_SPLIT
  return hipGetLastError();
}

hipError_t launch_scale_adjoint_split(const gswmtp_plan *p, bool honour_done, hipStream_t s) {
  const Dims &d = p->d;
  if (!p->scaled_adj || d.nf != d.Ur || d.Urp % kKB) return hipErrorInvalidValue;
  const size_t quads = (size_t)d.Rp * d.Urp / 4;
  const dim3 grid((unsigned)((quads + 255) / 256));
  const int *done = honour_done ? p->b.ctrl + CTRL_DONE : nullptr;
#define SCALE_ADJ(BF, NT)                                                                  \
  hipLaunchKernelGGL((k_scale_adjoint_split<BF, NT>), grid, dim3(256), 0, s, p->b.ob_r,    \
                     p->b.ob_i, p->b.theta_new, p->b.csr_foci, d.Ur, d.Rp, d.Urp, p->b.as_s, \
                     done)
  switch (p->precision) {
    case GSWMTP_BF16X3: SCALE_ADJ(true, 2); break;
    case GSWMTP_FP16X3: SCALE_ADJ(false, 2); break;
    case GSWMTP_BF16X6: SCALE_ADJ(true, 3); break;
    default: return hipErrorInvalidValue;
  }
#undef SCALE_ADJ
  return hipGetLastError();
}

size_t scatter_split_args_bytes() { return sizeof(ScatterSplitArgs); }

int fill_scatter_split_args(const gswmtp_plan *p, void *out) {
  const Dims &d = p->d;
  ScatterSplitArgs a{p->b.theta_new, p->b.wc_r, p->b.wc_i, p->b.csr_ic, p->b.csr_ptr,
                     p->b.csr_foci, p->b.ss, d.Ur, d.Urp, d.Cp, 1.f, p->b.ctrl + CTRL_DONE,
                     p->b.ob_r, p->b.ob_i, p->b.as_s, d.Rp, p->scaled_adj ? 1 : 0};
  std::memcpy(out, &a, sizeof a);
  if (p->scaled_adj) return (int)(((size_t)d.Rp * d.Urp / 4 + 255) / 256);
  return (d.Cp / 64) * (d.Urp / 32);
}

hipError_t launch_scatter_split_grouped(const void *items, const int *starts, int n, int blocks,
                                        int precision, hipStream_t s) {
  const ScatterSplitArgs *it = static_cast<const ScatterSplitArgs *>(items);
#define SCATTER_GROUPED(BF, NT)                                                                \
  hipLaunchKernelGGL((focus_scatter_split_grouped<BF, NT>), dim3(blocks), dim3(256), 0, s, it, \
                     starts, n)
  switch (precision) {
    case GSWMTP_BF16X3: SCATTER_GROUPED(true, 2); break;
    case GSWMTP_FP16X3: SCATTER_GROUPED(false, 2); break;
    case GSWMTP_BF16X6: SCATTER_GROUPED(true, 3); break;
    default: return hipErrorInvalidValue;
  }
#undef SCATTER_GROUPED
  return hipGetLastError();
}

hipError_t launch_gather_reduce(const gswmtp_plan *p, float *theta, float scale, hipStream_t s) {
  const int nf = p->d.nf;
  hipLaunchKernelGGL(gather_reduce, dim3((nf + 255) / 256), dim3(256), 0, s, p->b.gpart,
                     gather_partials(p), nf, gather_ld(p), scale, theta, nullptr, nullptr,
                     nullptr);
  return hipGetLastError();
}

hipError_t launch_field(const gswmtp_plan *p, hipStream_t s, float *field, float *intensity) {
  const Dims &d = p->d;
  const int nf = d.nf;
  const float scale = std::ldexp(1.f, -p->amp_exp);
  if (p->grid_form)   // straight from the dense grid (the forward skipped its gather)
    hipLaunchKernelGGL(grid_field, dim3((nf + 255) / 256), dim3(256), 0, s, p->b.g_r, p->b.g_i,
                       d.Ucp, d.axis == 0 ? p->b.iy : p->b.ix, d.axis == 0 ? p->b.ix : p->b.iy,
                       nf, scale, p->b.theta, p->b.intensity, field, intensity);
  else
    hipLaunchKernelGGL(gather_reduce, dim3((nf + 255) / 256), dim3(256), 0, s, p->b.gpart,
                       gather_partials(p), nf, gather_ld(p), scale, p->b.theta, p->b.intensity,
                       field, intensity);
  return hipGetLastError();
}

int gather_ld(const gswmtp_plan *p) { return (p->d.nf + 1) & ~1; }

int gather_partials(const gswmtp_plan *p) {
  return p->grid_form ? 1 : p->d.Cp / p->sched_fwd.tile.bn;
}

hipError_t launch_grid_gather(const gswmtp_plan *p, hipStream_t s) {
  const Dims &d = p->d;
  hipLaunchKernelGGL(grid_gather, dim3((d.nf + 255) / 256), dim3(256), 0, s, p->b.g_r, p->b.g_i,
                     d.Ucp, d.axis == 0 ? p->b.iy : p->b.ix, d.axis == 0 ? p->b.ix : p->b.iy,
                     d.nf, p->b.gpart);
  return hipGetLastError();
}

hipError_t launch_grid_scatter(const gswmtp_plan *p, const float *theta_new, float scale,
                               hipStream_t s, const float *g) {
  const Dims &d = p->d;
  hipLaunchKernelGGL(grid_scatter, dim3((d.nf + 255) / 256), dim3(256), 0, s, theta_new, scale,
                     d.axis == 0 ? p->b.iy : p->b.ix, d.axis == 0 ? p->b.ix : p->b.iy, d.nf,
                     p->b.tg_r, p->b.tg_i, d.Urp, g);
  return hipGetLastError();
}

static UpdateArgs update_args(const gswmtp_plan *p, int mode) {
  UpdateArgs a{};
  a.gpart = p->b.gpart;
  a.T = gather_partials(p);
  a.ldp = gather_ld(p);
  a.scale = std::ldexp(1.f, -p->amp_exp);
  a.theta = p->b.theta;
  a.theta_new = p->b.theta_new;
  a.intensity = p->b.intensity;
  a.target = p->b.target;
  a.tnorm = p->b.tnorm;
  a.tinv = p->b.tinv;
  a.tsqrt = p->b.tsqrt;
  a.w = p->b.w;
  a.fixph = p->b.fixph;
  a.stats = p->b.stats;
  a.hist = p->b.hist;
  a.ctrl = p->b.ctrl;
  a.s1 = p->b.upd_s1;
  a.s2 = p->b.upd_s2;
  a.snap = p->b.upd_snap;
  a.nwg = update_workgroups(p->d.nf);
  a.nf = p->d.nf;
  a.mode = mode;
  a.weighting = p->weighting;
  a.n_ap = (double)p->d.n_ap;
  a.sum_a2 = p->d.sum_a2;
  a.meas = p->meas_active;
  return a;
}

hipError_t launch_update(const gswmtp_plan *p, int mode, hipStream_t s) {
  const UpdateArgs a = update_args(p, mode);
  if (a.nwg == 0) {
    hipLaunchKernelGGL(focus_update, dim3(1), dim3(kUpdThreads), 0, s, a);
  } else {
    hipLaunchKernelGGL(focus_update_big<1>, dim3(a.nwg), dim3(kUpdThreads), 0, s, a);
    hipLaunchKernelGGL(focus_update_big<2>, dim3(a.nwg), dim3(kUpdThreads), 0, s, a);
    hipLaunchKernelGGL(focus_update_big<3>, dim3(a.nwg), dim3(kUpdThreads), 0, s, a);
  }
  return hipGetLastError();
}

size_t update_args_bytes() { return sizeof(UpdateArgs); }
int fill_update_args(const gswmtp_plan *p, int mode, int partials, void *out) {
  UpdateArgs a = update_args(p, mode);
  a.T = partials;   // partials per focus of the batch's forward product
  std::memcpy(out, &a, sizeof a);
  return a.nwg;
}
hipError_t launch_update_grouped(const GroupedUpdate &g, hipStream_t s) {
  const UpdateArgs *all = static_cast<const UpdateArgs *>(g.d_items);
  hipLaunchKernelGGL(focus_update_grouped<1>, dim3(g.blocks), dim3(kUpdThreads), 0, s, all,
                     g.d_starts, g.n_items);
  if (g.n_big > 0) {
    const UpdateArgs *big = static_cast<const UpdateArgs *>(g.d_big);
    hipLaunchKernelGGL(focus_update_grouped<2>, dim3(g.big_blocks), dim3(kUpdThreads), 0, s,
                       big, g.d_big_starts, g.n_big);
    hipLaunchKernelGGL(focus_update_grouped<3>, dim3(g.big_blocks), dim3(kUpdThreads), 0, s,
                       big, g.d_big_starts, g.n_big);
  }
  return hipGetLastError();
}

hipError_t launch_grad_field(const gswmtp_plan *p, const float *g, hipStream_t s) {
  hipLaunchKernelGGL(grad_field, dim3((p->d.nf + 255) / 256), dim3(256), 0, s, p->b.theta, g,
                     p->b.theta_new, p->d.nf);
  return hipGetLastError();
}

static ScatterArgs scatter_args(const gswmtp_plan *p, const float *theta_new, bool honour_done) {
  const Dims &d = p->d;
  ScatterArgs a{};
  a.tn = theta_new;
  a.wr = p->b.wc_r;
  a.wi = p->b.wc_i;
  a.ic = p->b.csr_ic;   // CSR order
  a.ptr = p->b.csr_ptr;
  a.foci = p->b.csr_foci;
  a.sr = p->b.s_r;
  a.si = p->b.s_i;
  a.Ur = d.Ur;
  a.Cp = d.Cp;
  a.done = honour_done ? p->b.ctrl + CTRL_DONE : nullptr;
  return a;
}

hipError_t launch_scatter(const gswmtp_plan *p, const float *theta_new, bool honour_done,
                          hipStream_t s) {
  const Dims &d = p->d;
  hipLaunchKernelGGL(focus_scatter, dim3((d.Cp + 1023) / 1024, d.Urp), dim3(256), 0, s,
                     scatter_args(p, theta_new, honour_done));
  return hipGetLastError();
}

size_t scatter_args_bytes() { return sizeof(ScatterArgs); }
int fill_scatter_args(const gswmtp_plan *p, void *out) {
  const ScatterArgs a = scatter_args(p, p->b.theta_new, true);
  std::memcpy(out, &a, sizeof a);
  return ((p->d.Cp + 1023) / 1024) * p->d.Urp;
}
hipError_t launch_scatter_grouped(const void *d_items, const int *d_starts, int n, int blocks,
                                  hipStream_t s) {
  hipLaunchKernelGGL(focus_scatter_grouped, dim3(blocks), dim3(256), 0, s,
                     static_cast<const ScatterArgs *>(d_items), d_starts, n);
  return hipGetLastError();
}

}  // namespace gswmtp
