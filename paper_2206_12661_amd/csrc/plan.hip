// C ABI, plan construction and the per-pass driver of the gfx950 GSW-MTP
// library (Liu et al., arXiv:2206.12661, Algorithm 1 with the matrix triple
// product of Eq. 2).
//
// Plan construction runs on the GPU: effective amplitude, compaction of the
// pupil to its non-zero rows/columns, the reduced focal grid (sorted unique
// focus coordinates per axis and the gather index of every focus), duplicate
// detection, the per-row focus lists used by the scatter, the kernel matrices
// (phase arguments reduced in float64), and E0 = A exp(i phi0).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <string>
#include <algorithm>
#include <utility>
#include <mutex>
#include <new>
#include <vector>

#include "adam_update.h"
#include "gswmtp_internal.h"

using namespace gswmtp;

namespace {

// ---------------------------------------------------------------------------
// Error handling
// ---------------------------------------------------------------------------

int fail(gswmtp_plan *p, int code, const char *what, hipError_t e = hipSuccess) {
  if (p) {
    char buf[512];
    if (e != hipSuccess)
      snprintf(buf, sizeof buf, "%s: %s (%s)", what, hipGetErrorString(e), hipGetErrorName(e));
    else
      snprintf(buf, sizeof buf, "%s", what);
    p->err = buf;
  }
  return code;
}

#define HIP_TRY(p, expr)                                       \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return fail((p), GSWMTP_E_HIP, #expr, e_); \
  } while (0)

// Keeps the plan's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
      changed = hipSetDevice(dev) == hipSuccess;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

// Orders plan work after the caller's stream and the caller after plan work.
hipError_t enter(gswmtp_plan *p) {
  hipError_t e = hipEventRecord(p->ev_user, p->user_stream);
  if (e != hipSuccess) return e;
  return hipStreamWaitEvent(p->stream, p->ev_user, 0);
}
hipError_t leave(gswmtp_plan *p) {
  hipError_t e = hipEventRecord(p->ev_int, p->stream);
  if (e != hipSuccess) return e;
  return hipStreamWaitEvent(p->user_stream, p->ev_int, 0);
}

size_t round_up(size_t v, size_t g) { return (v + g - 1) / g * g; }

// Bump allocator over one device allocation.
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(size_t count) {
    T *r = reinterpret_cast<T *>(base ? base + off : nullptr);
    off += round_up(count * sizeof(T) + 1, 256);
    return r;
  }
};

// Finite test by the exponent field (all ones: inf or NaN), branch-free over
// blocks of 4096 so that the loop vectorises; stops at the first bad block.
template <typename T, typename U, U kExp>
bool finite_bits(const T *a, size_t n) {
  for (size_t i0 = 0; i0 < n; i0 += 4096) {
    const size_t i1 = n - i0 < 4096 ? n : i0 + 4096;
    U bad = 0;
    for (size_t i = i0; i < i1; ++i) {
      U u;
      std::memcpy(&u, a + i, sizeof u);
      bad |= (U)((u & kExp) == kExp);
    }
    if (bad) return false;
  }
  return true;
}
bool finite_all(const double *a, size_t n) {
  return finite_bits<double, uint64_t, 0x7ff0000000000000ull>(a, n);
}
bool finite_all(const float *a, size_t n) { return finite_bits<float, uint32_t, 0x7f800000u>(a, n); }

// Valid amplitudes are finite and >= 0: bit patterns up to the largest
// finite float, and -0.0.
bool amplitude_ok(const float *a, size_t n) {
  for (size_t i0 = 0; i0 < n; i0 += 4096) {
    const size_t i1 = n - i0 < 4096 ? n : i0 + 4096;
    uint32_t bad = 0;
    for (size_t i = i0; i < i1; ++i) {
      uint32_t u;
      std::memcpy(&u, a + i, sizeof u);
      bad |= (uint32_t)(u > 0x7f7fffffu && u != 0x80000000u);
    }
    if (bad) return false;
  }
  return true;
}

// ---------------------------------------------------------------------------
// Plan-time kernels
// ---------------------------------------------------------------------------

// Effective amplitude: mask ? amplitude : 0 (in place).
__global__ void k_aeff(float *aeff, const unsigned char *mask, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && mask && !mask[i]) aeff[i] = 0.f;
}

__global__ void k_fill_f(float *a, float v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}
__global__ void k_fill_d(double *a, double v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// keep[r] = any(a[r * rs + c * cs] != 0 for c < len), one block per line.
__global__ void k_keep(const float *a, int lines, int len, size_t rs, size_t cs, int *keep) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const int r = blockIdx.x;
  int mine = 0;
  for (int c = threadIdx.x; c < len; c += blockDim.x)
    if (a[(size_t)r * rs + (size_t)c * cs] != 0.f) mine = 1;
  if (mine) atomicOr(&any, 1);
  __syncthreads();
  if (threadIdx.x == 0) keep[r] = any;
}

// Stable compaction of a 0/1 flag array: list[k] = index of the k-th set flag,
// pos[i] = k or -1; count written to *count.  One block of 1024 threads, each
// scanning a contiguous chunk.
__global__ __launch_bounds__(1024) void k_compact(const int *keep, int n, int *list, int *pos,
                                                  int *count) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int lo = t * chunk < n ? t * chunk : n;
  const int hi = lo + chunk < n ? lo + chunk : n;
  int c = 0;
  for (int i = lo; i < hi; ++i) c += keep[i] ? 1 : 0;
  part[t] = c;
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int q = 0; q < 1024; ++q) {
      const int v = part[q];
      part[q] = run;
      run += v;
    }
    *count = run;
  }
  __syncthreads();
  int k = part[t];
  for (int i = lo; i < hi; ++i) {
    if (keep[i]) {
      list[k] = i;
      pos[i] = k++;
    } else {
      pos[i] = -1;
    }
  }
}

// Aperture statistics: number of samples with A > 0 and sum of A^2 (float64).
// Workgroup b reduces the contiguous range [b chunk, (b + 1) chunk) with a
// fixed tree; one workgroup then sums the kApBlocks partials with a fixed
// tree, so the result depends on n alone, not on scheduling.
__global__ __launch_bounds__(256) void k_aperture_part(const float *a, size_t n, double *part,
                                                       int *cnt) {
  __shared__ double sd[256];
  __shared__ int si[256];
  const int t = threadIdx.x;
  const size_t chunk = (n + kApBlocks - 1) / kApBlocks;
  const size_t lo = (size_t)blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  double s = 0.0;
  int c = 0;
  for (size_t i = lo + t; i < hi; i += 256) {
    const double v = a[i];
    s += v * v;
    c += v > 0.0 ? 1 : 0;
  }
  sd[t] = s;
  si[t] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      sd[t] += sd[t + w];
      si[t] += si[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[blockIdx.x] = sd[0];
    cnt[blockIdx.x] = si[0];
  }
}

__global__ __launch_bounds__(kApBlocks) void k_aperture_sum(const double *part, const int *cnt,
                                                            int *n_ap, double *sum_a2) {
  __shared__ double sd[kApBlocks];
  __shared__ int si[kApBlocks];
  const int t = threadIdx.x;
  sd[t] = part[t];
  si[t] = cnt[t];
  __syncthreads();
  for (int w = kApBlocks / 2; w > 0; w >>= 1) {
    if (t < w) {
      sd[t] += sd[t + w];
      si[t] += si[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    *sum_a2 = sd[0];
    *n_ap = si[0];
  }
}

// Measured focus intensities (camera in the loop) divided by their sum, as
// the weight update normalises computed intensities: one workgroup, the sum
// in float64 in a fixed order.  The host has checked that the sum is > 0.
__global__ __launch_bounds__(1024) void k_meas_norm(double *m, int n) {
  __shared__ double part[1024];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) acc += m[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  const double sum = part[0];
  for (int i = threadIdx.x; i < n; i += 1024) m[i] = m[i] / sum;
}

// Column index of the focus at each CSR position (the scatter reads it
// beside the focus number instead of through it).
__global__ void k_csr_gather(const int *ic, const int *foci, int n, int *out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) out[p] = ic[foci[p]];
}

// Row pointers from the sorted order: ptr[a] = first sorted position whose
// row is >= a, ptr[ur] = n.
__global__ void k_row_ptr(const int *ir, const int *foci, int n, int ur, int *ptr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > n) return;
  const int prev = p > 0 ? ir[foci[p - 1]] : -1;
  const int cur = p < n ? ir[foci[p]] : ur;
  for (int a = prev + 1; a <= cur; ++a) ptr[a] = p;
}

// Target intensities normalised to unit sum (float64, fixed order).
// Unit-sum targets and the per-focus constants of the weight update:
// tnorm = target / sum, tinv = 1 / tnorm (0 where tnorm is 0), tsqrt =
// sqrt(target).  One workgroup, the sum in a fixed order.
__global__ __launch_bounds__(1024) void k_tnorm(const double *target, int n, double *tnorm,
                                                double *tinv, double *tsqrt) {
  __shared__ double s[1024];
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int i = t; i < n; i += 1024) acc += target[i];
  s[t] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) s[t] += s[t + w];
    __syncthreads();
  }
  const double tot = s[0];
  for (int i = t; i < n; i += 1024) {
    const double tn = target[i] / tot;
    tnorm[i] = tn;
    tinv[i] = tn > 0.0 ? 1.0 / tn : 0.0;
    tsqrt[i] = sqrt(target[i]);
  }
}

// exp(-2 pi i s c f) with the argument reduced exactly in float64:
// t = s c f, r = t - rint(t), then sincospi(-2 r).
// exp(-2 pi i s c f) exp(i pi z (s c)^2): the kernel phasor of Eq. 2 for
// sample coordinate c and focal coordinate f, times the defocus phase of a
// focus at axial position z (z = 0: the focal plane).  The phase in cycles
// is reduced to [-1/2, 1/2] in float64 before sincospi.
__device__ __forceinline__ void kernel_phasor(double s, double c, double f, double z, float *re,
                                              float *im) {
  const double sc = s * c;
  const double t = sc * f - 0.5 * z * sc * sc;
  const double r = t - rint(t);
  double sn, cs;
  sincospi(-2.0 * r, &sn, &cs);
  *re = (float)cs;
  *im = (float)sn;
}

// Omega_r in both layouts: OmT[j][a] and OmC[a][j] = conj(OmT[j][a]).
__global__ void k_omega_r(const double *coord, const int *kept, int Rk, const double *fu,
                          const double *fuz, int Ur, double s, int Rp, int Urp, float *omt_r,
                          float *omt_i, float *omc_r, float *omc_i) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)Rp * Urp) return;
  const int j = (int)(id / Urp), a = (int)(id % Urp);
  float re = 0.f, im = 0.f;
  if (j < Rk && a < Ur) kernel_phasor(s, coord[kept[j]], fu[a], fuz[a], &re, &im);
  omt_r[(size_t)j * Urp + a] = re;
  omt_i[(size_t)j * Urp + a] = im;
  omc_r[(size_t)a * Rp + j] = re;
  omc_i[(size_t)a * Rp + j] = -im;
}

// Wc[b][i] = exp(-2 pi i s_c uc_i C_b) for b < Uc, i < Cp (0 past Ck).
// Grid form tables: Omega_c transposed ([Cp][Ucp], B operand of the grid
// product) and the negated imaginary plane of Omega_c^T ([Ucp][Cp], with the
// real plane the conjugate, B operand of the scatter product).  Rows and
// columns past Uc stay zero.
__global__ void k_grid_tables(const float *wr, const float *wi, int Uc, int Cp, int Ucp,
                              float *wt_r, float *wt_i, float *wn_i) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)Ucp * Cp) return;
  const int b = (int)(id / Cp), i = (int)(id % Cp);
  const float re = b < Uc ? wr[(size_t)b * Cp + i] : 0.f;
  const float im = b < Uc ? wi[(size_t)b * Cp + i] : 0.f;
  wt_r[(size_t)i * Ucp + b] = re;
  wt_i[(size_t)i * Ucp + b] = im;
  wn_i[id] = -im;
}

__global__ void k_omega_c(const double *coord, const int *kept, int Ck, const double *fu,
                          const double *fuz, int Uc, double s, int Cp, float *wr, float *wi) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)Uc * Cp) return;
  const int b = (int)(id / Cp), i = (int)(id % Cp);
  float re = 0.f, im = 0.f;
  if (i < Ck) kernel_phasor(s, coord[kept[i]], fu[b], fuz[b], &re, &im);
  wr[id] = re;
  wi[id] = im;
}

// Map an internal (r, c) sample to the user's (y, x); false in the padding.
struct Orient {
  const int *rows, *cols;
  int axis, Rk, Ck;
  __device__ bool user(int r, int c, int *y, int *x) const {
    if (r >= Rk || c >= Ck) return false;
    if (axis == 0) {
      *y = rows[r];
      *x = cols[c];
    } else {
      *y = rows[c];
      *x = cols[r];
    }
    return true;
  }
};

// Internal amplitude times an exact power-of-two scale (zero in the padding).
__global__ void k_encode_amp(Orient o, const float *aeff, float scale, int nx, int Rp, int Cp,
                             float *amp) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)Rp * Cp) return;
  int y, x;
  amp[id] = o.user((int)(id / Cp), (int)(id % Cp), &y, &x) ? aeff[(size_t)y * nx + x] * scale
                                                            : 0.f;
}

// Pupil field E = A exp(i phi) from a user-layout phase (nullable = zeros);
// ctrl (nullable): the recorded focal phases of phase fixing are dropped
// (its flag cleared by the first thread), as a new phase requires.
__global__ void k_encode_phase(Orient o, const float *phi, const float *amp, int nx, int Rp,
                               int Cp, float *pr, float *pi, int *ctrl) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ctrl && id == 0) ctrl[CTRL_FIXED] = 0;
  if (id >= (size_t)Rp * Cp) return;
  int y, x;
  float re = 0.f, im = 0.f;
  if (o.user((int)(id / Cp), (int)(id % Cp), &y, &x)) {
    const float a = amp[id];
    const float ph = phi ? phi[(size_t)y * nx + x] : 0.f;
    float s, c;
    sincosf(ph, &s, &c);
    re = a * c;
    im = a * s;
  }
  pr[id] = re;
  pi[id] = im;
}

// User-layout complex field (interleaved) -> internal planes (zero padding).
__global__ void k_compact_complex(Orient o, const float *in, int nx, int Rp, int Cp, float *xr,
                                  float *xi) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)Rp * Cp) return;
  int y, x;
  float re = 0.f, im = 0.f;
  if (o.user((int)(id / Cp), (int)(id % Cp), &y, &x)) {
    re = in[2 * ((size_t)y * nx + x)];
    im = in[2 * ((size_t)y * nx + x) + 1];
  }
  xr[id] = re;
  xi[id] = im;
}

// Internal (r, c) of a user (y, x), or false when the sample was compacted away.
__device__ __forceinline__ bool internal_of(const int *row_pos, const int *col_pos, int axis,
                                            int y, int x, int *r, int *c) {
  const int rp = row_pos[y], cp = col_pos[x];
  if (rp < 0 || cp < 0) return false;
  *r = axis == 0 ? rp : cp;
  *c = axis == 0 ? cp : rp;
  return true;
}

// Phase of the current pupil field in the user's layout: atan2 on aperture
// samples, (-pi, pi]; 0 outside the aperture.
__global__ void k_phase_out(const float *pr, const float *pi, const float *amp,
                            const int *row_pos, const int *col_pos, int axis, int ny, int nx,
                            int Cp, float *out) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)ny * nx) return;
  const int y = (int)(id / nx), x = (int)(id % nx);
  int r, c;
  float ph = 0.f;
  if (internal_of(row_pos, col_pos, axis, y, x, &r, &c)) {
    const size_t o = (size_t)r * Cp + c;
    if (amp[o] > 0.f) {
      ph = atan2f(pi[o], pr[o]);
      if (ph == -3.14159274101257324f) ph = 3.14159274101257324f;
    }
  }
  out[id] = ph;
}

// Internal planes -> user-layout interleaved complex (zero where compacted).
__global__ void k_expand_complex(const float *xr, const float *xi, const int *row_pos,
                                 const int *col_pos, int axis, int ny, int nx, int Cp,
                                 float scale, float *out) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)ny * nx) return;
  int r, c;
  float re = 0.f, im = 0.f;
  if (internal_of(row_pos, col_pos, axis, (int)(id / nx), (int)(id % nx), &r, &c)) {
    re = xr[(size_t)r * Cp + c] * scale;
    im = xi[(size_t)r * Cp + c] * scale;
  }
  out[2 * id] = re;
  out[2 * id + 1] = im;
}

// Adam on user-layout phases (adam_update.h) with the gradient read from the
// internal real plane in place (0 where compacted): the expansion of
// k_expand_real and the update of the library's Adam kernel in one pass.
// Grid-stride over groups of VEC values (VEC = 4: 16-byte accesses of phi, m
// and v, which the caller has checked are aligned and a multiple of 4 long).
__device__ __forceinline__ float internal_value(const float *xr, const int *row_pos,
                                                const int *col_pos, int axis, int nx, int Cp,
                                                size_t id) {
  int r, c;
  if (internal_of(row_pos, col_pos, axis, (int)(id / nx), (int)(id % nx), &r, &c))
    return xr[(size_t)r * Cp + c];
  return 0.f;
}

template <int VEC>
__global__ __launch_bounds__(256) void k_adam_internal(const float *xr, const int *row_pos,
                                                       const int *col_pos, int axis, int ny,
                                                       int nx, int Cp, float *phi, float *m,
                                                       float *v, const float *step, float lr,
                                                       float b1, float b2, float eps) {
  float step_size, rbc2;
  adam_scalars(*step, lr, b1, b2, step_size, rbc2);
  const size_t n = (size_t)ny * nx / VEC;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    if constexpr (VEC == 4) {
      float4 p = reinterpret_cast<float4 *>(phi)[i], mi = reinterpret_cast<float4 *>(m)[i],
             vi = reinterpret_cast<float4 *>(v)[i];
      const size_t id = 4 * i;
      adam_apply(p.x, mi.x, vi.x, internal_value(xr, row_pos, col_pos, axis, nx, Cp, id), b1,
                 b2, step_size, rbc2, eps);
      adam_apply(p.y, mi.y, vi.y, internal_value(xr, row_pos, col_pos, axis, nx, Cp, id + 1),
                 b1, b2, step_size, rbc2, eps);
      adam_apply(p.z, mi.z, vi.z, internal_value(xr, row_pos, col_pos, axis, nx, Cp, id + 2),
                 b1, b2, step_size, rbc2, eps);
      adam_apply(p.w, mi.w, vi.w, internal_value(xr, row_pos, col_pos, axis, nx, Cp, id + 3),
                 b1, b2, step_size, rbc2, eps);
      reinterpret_cast<float4 *>(phi)[i] = p;
      reinterpret_cast<float4 *>(m)[i] = mi;
      reinterpret_cast<float4 *>(v)[i] = vi;
    } else {
      float p = phi[i], mi = m[i], vi = v[i];
      adam_apply(p, mi, vi, internal_value(xr, row_pos, col_pos, axis, nx, Cp, i), b1, b2,
                 step_size, rbc2, eps);
      phi[i] = p;
      m[i] = mi;
      v[i] = vi;
    }
  }
}

// Internal real plane -> user layout (zero where compacted).
__global__ void k_expand_real(const float *xr, const int *row_pos, const int *col_pos, int axis,
                              int ny, int nx, int Cp, float *out) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)ny * nx) return;
  int r, c;
  float v = 0.f;
  if (internal_of(row_pos, col_pos, axis, (int)(id / nx), (int)(id % nx), &r, &c))
    v = xr[(size_t)r * Cp + c];
  out[id] = v;
}


// ---- split-precision layouts (16-bit term planes, k-contiguous) ----

// Omega_r as split planes (k-blocked): forward A [re/im][term] x [Urp][Rp]
// and adjoint A = Omega_r^H [re/im][term] x [Rp][Urp].
template <bool BF, int NT>
__global__ void k_omega_r_split(const double *coord, const int *kept, int Rk, const double *fu,
                                const double *fuz, int Ur, double s, int Rp, int Urp,
                                unsigned short *af, unsigned short *ab, float *obr, float *obi) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)Rp * Urp) return;
  const int j = (int)(id / Urp), a = (int)(id % Urp);
  float re = 0.f, im = 0.f;
  if (j < Rk && a < Ur) kernel_phasor(s, coord[kept[j]], fu[a], fuz[a], &re, &im);
  unsigned short tr[NT], ti[NT], tc[NT];
  split_terms<BF, NT>(re, tr, 1);
  split_terms<BF, NT>(im, ti, 1);
  split_terms<BF, NT>(-im, tc, 1);
  const size_t plane = (size_t)Rp * Urp;
  const size_t of = kblk_index(a, j, Urp), ob = kblk_index(j, a, Rp);
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    af[(size_t)q * plane + of] = tr[q];
    af[(size_t)(NT + q) * plane + of] = ti[q];
    ab[(size_t)q * plane + ob] = tr[q];
    ab[(size_t)(NT + q) * plane + ob] = tc[q];
  }
  if (obr) {   // the float32 values the planes split, for the scaled adjoint
    obr[ob] = re;
    obi[ob] = -im;
  }
}

__global__ void k_fill_unit(float *t, int nf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  t[2 * i] = 1.f;
  t[2 * i + 1] = 0.f;
}

// Pupil field from a phase as split planes P^T [re/im][term] x [Cp][Rp]
// (k-blocked)
// (amp already carries the power-of-two scale).
template <bool BF, int NT>
__global__ void k_encode_phase_split(Orient o, const float *phi, const float *amp, int nx,
                                     int Rp, int Cp, unsigned short *pt, int *ctrl) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ctrl && id == 0) ctrl[CTRL_FIXED] = 0;
  if (id >= (size_t)Rp * Cp) return;
  const int i = (int)(id / Rp), j = (int)(id % Rp);
  int y, x;
  float re = 0.f, im = 0.f;
  if (o.user(j, i, &y, &x)) {
    const float a = amp[(size_t)j * Cp + i];
    const float ph = phi ? phi[(size_t)y * nx + x] : 0.f;
    float sn, cs;
    sincosf(ph, &sn, &cs);
    re = a * cs;
    im = a * sn;
  }
  const size_t plane = (size_t)Rp * Cp, at = kblk_index(i, j, Cp);
  split_terms<BF, NT>(re, pt + at, (int)plane);
  split_terms<BF, NT>(im, pt + (size_t)NT * plane + at, (int)plane);
}

// User-layout complex field (interleaved), times scale, as split planes P^T.
template <bool BF, int NT>
__global__ void k_compact_split(Orient o, const float *in, float scale, int nx, int Rp, int Cp,
                                unsigned short *pt) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)Rp * Cp) return;
  const int i = (int)(id / Rp), j = (int)(id % Rp);
  int y, x;
  float re = 0.f, im = 0.f;
  if (o.user(j, i, &y, &x)) {
    re = in[2 * ((size_t)y * nx + x)] * scale;
    im = in[2 * ((size_t)y * nx + x) + 1] * scale;
  }
  const size_t plane = (size_t)Rp * Cp, at = kblk_index(i, j, Cp);
  split_terms<BF, NT>(re, pt + at, (int)plane);
  split_terms<BF, NT>(im, pt + (size_t)NT * plane + at, (int)plane);
}

// Phase of the split pupil planes in the user's layout.
__global__ void k_phase_out_split(const unsigned short *pt, bool bf, int nt, const float *amp,
                                  const int *row_pos, const int *col_pos, int axis, int ny,
                                  int nx, int Rp, int Cp, float *out) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)ny * nx) return;
  const int y = (int)(id / nx), x = (int)(id % nx);
  int r, c;
  float ph = 0.f;
  if (internal_of(row_pos, col_pos, axis, y, x, &r, &c) && amp[(size_t)r * Cp + c] > 0.f) {
    const size_t plane = (size_t)Rp * Cp, o = kblk_index(c, r, Cp);
    const float re = join_terms(bf, nt, pt + o, plane);
    const float im = join_terms(bf, nt, pt + (size_t)nt * plane + o, plane);
    ph = atan2f(im, re);
    if (ph == -3.14159274101257324f) ph = 3.14159274101257324f;
  }
  out[id] = ph;
}

#define DISPATCH_SPLIT(prec, X)          \
  switch (prec) {                        \
    case GSWMTP_BF16X3: X(true, 2); break; \
    case GSWMTP_FP16X3: X(false, 2); break; \
    case GSWMTP_BF16X6: X(true, 3); break; \
    default: break;                      \
  }

// Run control written by a kernel (graph-safe, no memset): clear the done
// flag and set the termination threshold.
__global__ void k_control(int *ctrl, double *stats, double stop) {
  ctrl[CTRL_DONE] = 0;
  ctrl[CTRL_NONFINITE] = 0;
  stats[ST_STOP] = stop;
}

__global__ void k_set_state(int *ctrl, int iters) {
  ctrl[CTRL_ITERS] = iters;
  ctrl[CTRL_HIST] = 0;
  ctrl[CTRL_DONE] = 0;
  ctrl[CTRL_FIXED] = 0;
}

// Phase fixing from updating pass `from` on (0: off); frozen phasors are
// recorded afresh by the next pass that uses them.
__global__ void k_set_fix(int *ctrl, int from) {
  ctrl[CTRL_FIX] = from;
  ctrl[CTRL_FIXED] = 0;
}

inline dim3 grid1(size_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

Orient orient_of(const gswmtp_plan *p) {
  Orient o;
  o.rows = p->b.rows;
  o.cols = p->b.cols;
  o.axis = p->d.axis;
  o.Rk = p->d.Rk;
  o.Ck = p->d.Ck;
  return o;
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------

int validate(const gswmtp_desc *d) {
  if (!d) return GSWMTP_E_INVAL;
  if (d->ny < 1 || d->nx < 1 || d->ny > kMaxSide || d->nx > kMaxSide) return GSWMTP_E_INVAL;
  if (d->n_foci < 1 || d->n_foci > kMaxFoci) return GSWMTP_E_INVAL;
  if (!d->fx || !d->fy || !d->target) return GSWMTP_E_INVAL;
  if (!std::isfinite(d->s_x) || !std::isfinite(d->s_y) || d->s_x == 0.0 || d->s_y == 0.0)
    return GSWMTP_E_INVAL;
  if (d->precision < GSWMTP_FP32 || d->precision > GSWMTP_BF16X6) return GSWMTP_E_INVAL;
  if (d->axis < -1 || d->axis > 1) return GSWMTP_E_INVAL;
  if (d->weighting < GSWMTP_WEIGHT_GSW || d->weighting > GSWMTP_WEIGHT_GS) return GSWMTP_E_INVAL;
  const size_t nf = (size_t)d->n_foci, np = (size_t)d->ny * d->nx;
  if (!finite_all(d->fx, nf) || !finite_all(d->fy, nf) || !finite_all(d->target, nf))
    return GSWMTP_E_INVAL;
  if (d->fz && !finite_all(d->fz, nf)) return GSWMTP_E_INVAL;
  double tsum = 0.0;
  for (size_t i = 0; i < nf; ++i) {
    if (d->target[i] < 0.0) return GSWMTP_E_INVAL;
    tsum += d->target[i];
  }
  if (!(tsum > 0.0) || !std::isfinite(tsum)) return GSWMTP_E_INVAL;
  if (d->u && !finite_all(d->u, d->nx)) return GSWMTP_E_INVAL;
  if (d->v && !finite_all(d->v, d->ny)) return GSWMTP_E_INVAL;
  if (d->amplitude && !amplitude_ok(d->amplitude, np)) return GSWMTP_E_INVAL;
  if (d->phi0 && !finite_all(d->phi0, np)) return GSWMTP_E_INVAL;
  return GSWMTP_OK;
}

int check_device(gswmtp_plan *p) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return fail(p, GSWMTP_E_NODEV, "no HIP device");
  HIP_TRY(p, hipGetDevice(&p->device));
  hipDeviceProp_t prop;
  HIP_TRY(p, hipGetDeviceProperties(&prop, p->device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(p, GSWMTP_E_NODEV, "device is not gfx950");
  p->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  return GSWMTP_OK;
}

void free_plan(gswmtp_plan *p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  if (p->graph1) (void)hipGraphExecDestroy(p->graph1);
  if (p->graph8) (void)hipGraphExecDestroy(p->graph8);
  if (!p->ws) {   // a caller's workspace is the caller's to free
    if (p->pool0) (void)hipFree(p->pool0);
    if (p->pool1) (void)hipFree(p->pool1);
  }
  for (auto &e : p->ev_t)
    if (e) (void)hipEventDestroy(e);
  if (p->ev_user) (void)hipEventDestroy(p->ev_user);
  if (p->ev_int) (void)hipEventDestroy(p->ev_int);
  if (p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

// GEMM tile per product.  float32: 64 x 64 complex tiles, 16 k per stage
// (three workgroups per CU resident).  Split modes: 64 x 64 tiles with 32 k
// per stage (16-bit operands need longer stages to cover load latency) and
// the software-pipelined stage loop (two-term modes, 64 x 128 tiles where
// they fill one round of workgroups) or two k-groups (three-term).  GSWMTP_SPLIT_LOOP=pipe|kg2|plain picks
// the split products' loop (kg2: each stage's two k-steps taken by two
// groups of four waves); GSWMTP_TILE=BMxBN[xBK] overrides the tile (BK only
// for split modes; other tiles use the plain loop).
GemmTile choose_tile(int M, int N, bool split, int terms = 2, int cus = 256) {
  GemmTile t{64, 64, split ? 32 : 16, 1, 0};
  // three-term operands hold too many fragment registers to pipeline them at
  // two workgroups per CU: two k-groups instead; two-term 64 x 128 tiles take
  // the direct loop (B straight into registers, ~3% faster than pipe there)
  const char *lp = std::getenv("GSWMTP_SPLIT_LOOP");
  const std::string v = lp ? lp : terms > 2 ? "kg2" : "direct";
  if (split) {
    t.kg = v == "kg2" ? 2 : 1;
    t.pipe = v == "pipe" || v == "direct" ? 1 : 0;
    // 64 x 128 tiles (one workgroup per CU, a quarter fewer LDS and L2 bytes
    // per MFMA) when they fill at least half of the CUs in one round and do
    // not spill into a second
    const long wide = (long)(M / 64) * (N / 128);
    if (t.pipe && N % 128 == 0 && wide <= cus && 2 * wide >= cus) t.bn = 128;
  }
  const char *env = std::getenv("GSWMTP_TILE");
  if (env) {
    int bm = 0, bn = 0, bk = 0;
    const int n = std::sscanf(env, "%dx%dx%d", &bm, &bn, &bk);
    if (n >= 2 && (bm == 64 || bm == 128) && (bn == 64 || bn == 128) && M % bm == 0 &&
        N % bn == 0) {
      t.bm = bm;
      t.bn = bn;
      if (split && n == 3 && (bk == 16 || bk == 32)) t.bk = bk;
      if (t.bk != 32 || (t.bm == 128 && t.bn == 128)) t.kg = 1, t.pipe = 0;
      if (t.bm != 64 || t.bn != 64) t.kg = 1;
    }
  }
  if (split && v == "direct" && t.pipe && t.bm == 64 && t.bn == 128 && t.bk == 32 &&
      terms == 2)
    t.pipe = 2;
  return t;
}

bool split_enabled() {
  const char *env = std::getenv("GSWMTP_NO_SPLITK");
  return !(env && std::atoi(env) != 0);
}

bool is_split(const gswmtp_plan *p) { return split_terms_of(p->precision) > 0; }

// Stages of one pass, in either arithmetic.
// Forward product with the focus gather fused into its epilogue (partials
// reduced by the focus update).
// Float32 forward products for a compacted pupil field (er, ei) [Rp][Cp],
// leaving Theta's gather partials: the gather form (second product at the
// foci, in the first product's epilogue) or the grid form (L^T = P^T
// Omega_r^T, then G = L Omega_c^T on the matrix cores, then Theta_n = G at
// the focus).
// Split grid form, forward: L^T = P^T Omega_r^T on the 16-bit matrix cores
// (pt: the split planes of P^T), then the float32 grid product and gather.
hipError_t split_grid_forward(gswmtp_plan *p, const unsigned short *pt, bool done,
                              hipStream_t s, bool gather = true) {
  const Dims &D = p->d;
  Bufs &b = p->b;
  hipError_t e = launch_cgemm_split_ex(p, p->sched_f1, pt, D.Cp, b.as_f, D.Urp, D.Rp, b.lt_r,
                                       b.lt_i, D.Urp, done, s);
  if (e != hipSuccess) return e;
  e = launch_cgemm_ex(p, p->sched_f2, b.lt_r, b.lt_i, D.Urp, b.wt_r, b.wt_i, D.Ucp, b.g_r, b.g_i,
                      D.Ucp, D.Urp, D.Ucp, D.Cp, EPI_STORE, done, s);
  if (e != hipSuccess || !gather) return e;
  return launch_grid_gather(p, s);
}

// gather = false (grid form only): leave the dense grid G without gathering
// the foci from it (launch_field reads them from G).
hipError_t forward_products(gswmtp_plan *p, const float *er, const float *ei, bool done,
                            hipStream_t s, bool gather = true) {
  if (!p->grid_form)
    return launch_cgemm(p, true, EPI_GATHER, er, ei, nullptr, nullptr, nullptr, nullptr, done, s);
  const Dims &D = p->d;
  Bufs &b = p->b;
  hipError_t e = launch_cgemm_ex(p, p->sched_f1, er, ei, D.Cp, b.omt_r, b.omt_i, D.Urp, b.lt_r,
                                 b.lt_i, D.Urp, D.Cp, D.Urp, D.Rp, EPI_STORE, done, s);
  if (e != hipSuccess) return e;
  e = launch_cgemm_ex(p, p->sched_f2, b.lt_r, b.lt_i, D.Urp, b.wt_r, b.wt_i, D.Ucp, b.g_r, b.g_i,
                      D.Ucp, D.Urp, D.Ucp, D.Cp, EPI_STORE, done, s);
  if (e != hipSuccess || !gather) return e;
  return launch_grid_gather(p, s);
}

// Float32 scatter of focal values theta (device, interleaved) into S: per
// row of foci (gather form) or as the product Theta'_grid conj(Omega_c)
// (grid form).
hipError_t scatter_products(gswmtp_plan *p, const float *theta, bool done, hipStream_t s,
                            float scale = 1.f, const float *g = nullptr) {
  if (!p->grid_form) return launch_scatter(p, theta, done, s);
  const Dims &D = p->d;
  Bufs &b = p->b;
  hipError_t e = launch_grid_scatter(p, theta, scale, s, g);
  if (e != hipSuccess) return e;
  return launch_cgemm_ex(p, p->sched_a1, b.tg_r, b.tg_i, D.Urp, b.wc_r, b.wn_i, D.Cp, b.s_r,
                         b.s_i, D.Cp, D.Urp, D.Cp, D.Ucp, EPI_STORE, done, s);
}

// Split grid form, scatter: the float32 grid scatter product into S, then S
// as the split planes of S^T for the adjoint product.
hipError_t split_grid_scatter(gswmtp_plan *p, const float *theta, float scale, bool done,
                              hipStream_t s) {
  hipError_t e = scatter_products(p, theta, done, s, scale);
  if (e != hipSuccess) return e;
  return launch_split_transpose(p, p->b.s_r, p->b.s_i, 1.f, done, s);
}

// gather = false: the grid form leaves the focus gather to launch_field.
hipError_t stage_forward(gswmtp_plan *p, bool done, hipStream_t s, bool gather = true) {
  if (is_split(p) && p->grid_form) return split_grid_forward(p, p->b.ps, done, s, gather);
  if (is_split(p))
    return launch_cgemm_split(p, true, EPI_GATHER, p->b.ps, nullptr, nullptr, nullptr, done, s);
  return forward_products(p, p->b.p_r, p->b.p_i, done, s, gather);
}
hipError_t stage_scatter(gswmtp_plan *p, bool done, hipStream_t s) {
  if (p->scaled_adj) return launch_scale_adjoint_split(p, done, s);
  if (is_split(p) && p->grid_form) return split_grid_scatter(p, p->b.theta_new, 1.f, done, s);
  if (is_split(p)) return launch_scatter_split(p, p->b.theta_new, 1.f, done, s);
  return scatter_products(p, p->b.theta_new, done, s);
}
// phases: 1 the product launch, 2 its split-K tail launch, 3 both.
hipError_t stage_adjoint(gswmtp_plan *p, bool done, hipStream_t s, int phases = 3) {
  if (p->scaled_adj)
    return launch_cgemm_split(p, false, EPI_PROJECT, p->b.bs, nullptr, nullptr, p->b.ps, done, s,
                              phases, p->b.as_s);
  if (is_split(p))
    return launch_cgemm_split(p, false, EPI_PROJECT, p->b.ss, nullptr, nullptr, p->b.ps, done, s,
                              phases);
  return launch_cgemm(p, false, EPI_PROJECT, p->b.s_r, p->b.s_i, p->b.p_r, p->b.p_i, nullptr,
                      nullptr, done, s, phases);
}

// One GSW pass (Algorithm 1 from forward propagation to the projected pupil).
hipError_t enqueue_pass(gswmtp_plan *p, hipStream_t s) {
  hipError_t e;
  if ((e = stage_forward(p, true, s)) != hipSuccess) return e;
  if ((e = launch_update(p, UPD_ITERATE, s)) != hipSuccess) return e;
  if ((e = stage_scatter(p, true, s)) != hipSuccess) return e;
  return stage_adjoint(p, true, s);
}

// Forward field and statistics of the current phase (no weight update).
// Forward of the current phase (lazy): theta and intensity, and with stats
// the focus statistics too.  The statistics are recomputed from a forward of
// their own when asked for after a field-only call (the gather partials may
// have been reused by an operator call since).
hipError_t ensure_forward(gswmtp_plan *p, bool stats) {
  if (stats ? p->stats_valid : p->fwd_valid) return hipSuccess;
  hipError_t e;
  if ((e = stage_forward(p, false, p->stream, stats)) != hipSuccess) return e;
  if (stats) {
    if ((e = launch_update(p, UPD_STATS, p->stream)) != hipSuccess) return e;
    p->stats_valid = true;
  } else if ((e = launch_field(p, p->stream)) != hipSuccess) {
    return e;
  }
  p->fwd_valid = true;
  return hipSuccess;
}

// Encode a user-layout phase (device, nullable = zeros) into the pupil field;
// clear_fixed: also drop the recorded focal phases of phase fixing.
hipError_t encode_phase(gswmtp_plan *p, const float *dev_phi, hipStream_t s, bool clear_fixed) {
  int *ctrl = clear_fixed ? p->b.ctrl : nullptr;
  const Dims &D = p->d;
  const Orient o = orient_of(p);
  const dim3 g = grid1((size_t)D.Rp * D.Cp);
  if (is_split(p)) {
#define ENC(BF, NT)                                                                              \
  hipLaunchKernelGGL((k_encode_phase_split<BF, NT>), g, dim3(256), 0, s, o, dev_phi, p->b.amp, \
                     D.nx, D.Rp, D.Cp, p->b.ps, ctrl)
    DISPATCH_SPLIT(p->precision, ENC)
#undef ENC
  } else {
    hipLaunchKernelGGL(k_encode_phase, g, dim3(256), 0, s, o, dev_phi, p->b.amp, D.nx, D.Rp,
                       D.Cp, p->b.p_r, p->b.p_i, ctrl);
  }
  return hipGetLastError();
}

// Phase of the current pupil field into device memory (user layout).
hipError_t phase_out(gswmtp_plan *p, float *dev_out, hipStream_t s) {
  const Dims &D = p->d;
  const dim3 g = grid1((size_t)D.ny * D.nx);
  if (is_split(p)) {
    hipLaunchKernelGGL(k_phase_out_split, g, dim3(256), 0, s, p->b.ps,
                       split_is_bf16(p->precision), split_terms_of(p->precision), p->b.amp,
                       p->b.row_pos, p->b.col_pos, D.axis, D.ny, D.nx, D.Rp, D.Cp, dev_out);
  } else {
    hipLaunchKernelGGL(k_phase_out, g, dim3(256), 0, s, p->b.p_r, p->b.p_i, p->b.amp,
                       p->b.row_pos, p->b.col_pos, D.axis, D.ny, D.nx, D.Cp, dev_out);
  }
  return hipGetLastError();
}

// Exponent e with max|v| * 2^e in [0.5, 1) (0 for an all-zero input).
int scale_exponent(double amax) {
  if (!(amax > 0.0) || !std::isfinite(amax)) return 0;
  return -std::ilogb(amax) - 1;
}

hipError_t capture(gswmtp_plan *p, int passes, hipGraphExec_t *out) {
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t le = hipSuccess;
  for (int i = 0; i < passes && le == hipSuccess; ++i) le = enqueue_pass(p, p->stream);
  e = hipStreamEndCapture(p->stream, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return le;
  }
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

// Pool 0 (inputs, index work, per-focus state): every buffer carved in a
// fixed order from a bump allocator (a null base only measures).
void carve_pool0(Carver &c, Bufs &b, size_t nf, size_t ny, size_t nx) {
  const size_t np = ny * nx;
  b.fx = c.take<double>(nf); b.fy = c.take<double>(nf); b.fz = c.take<double>(nf);
  b.xzu = c.take<double>(nf); b.yzu = c.take<double>(nf); b.meas = c.take<double>(nf);
  b.target = c.take<double>(nf); b.tnorm = c.take<double>(nf);
  b.tinv = c.take<double>(nf); b.tsqrt = c.take<double>(nf);
  b.xu = c.take<double>(nf); b.yu = c.take<double>(nf);
  b.ix = c.take<int>(nf); b.iy = c.take<int>(nf);
  b.skey0 = c.take<uint64_t>(nf); b.skey1 = c.take<uint64_t>(nf);
  b.sval0 = c.take<int>(nf); b.sval1 = c.take<int>(nf);
  b.shist = c.take<int>(index_hist_ints((int)nf));
  b.shead = c.take<int>(nf); b.srank = c.take<int>(nf);
  b.rows = c.take<int>(ny); b.row_pos = c.take<int>(ny); b.keep_row = c.take<int>(ny);
  b.cols = c.take<int>(nx); b.col_pos = c.take<int>(nx); b.keep_col = c.take<int>(nx);
  b.aeff = c.take<float>(np);
  b.ucoord = c.take<double>(nx); b.vcoord = c.take<double>(ny);
  b.csr_foci = c.take<int>(nf); b.csr_ptr = c.take<int>(nf + 1); b.csr_ic = c.take<int>(nf);
  b.csr_ir = c.take<int>(nf);
  b.scalars = c.take<int>(16); b.dscalars = c.take<double>(8); b.dup = c.take<int>(1);
  b.ap_part = c.take<double>(kApBlocks); b.ap_cnt = c.take<int>(kApBlocks);
  b.theta = c.take<float>(2 * nf); b.theta_new = c.take<float>(2 * nf);
  b.intensity = c.take<float>(nf);
  b.w = c.take<double>(nf); b.stats = c.take<double>(ST_N); b.fixph = c.take<double>(2 * nf);
  b.upd_s1 = c.take<double>((nf + kUpdThreads - 1) / kUpdThreads);
  b.upd_s2 = c.take<double>(5 * ((nf + kUpdThreads - 1) / kUpdThreads));
  b.upd_snap = c.take<int>(8);
  b.hist = c.take<double>(3 * (size_t)kHistCap); b.ctrl = c.take<int>(CTRL_N);
  b.iobuf = c.take<float>(2 * np);
}

// The sizes and schedules that follow from the index counts (unique focal
// coordinates, kept pupil rows and columns) and the descriptor: the axis,
// the padded product sizes, the product schedules and the form of the
// second product.
void derive_layout(gswmtp_plan *p, const gswmtp_desc *d) {
  Dims &D = p->d;
  D.axis = d->axis >= 0 ? d->axis : (D.ux < D.uy ? 1 : 0);
  if (D.axis == 0) {
    D.Rk = D.ny_kept; D.Ck = D.nx_kept; D.Ur = D.uy; D.Uc = D.ux;
  } else {
    D.Rk = D.nx_kept; D.Ck = D.ny_kept; D.Ur = D.ux; D.Uc = D.uy;
  }
  D.Rp = (int)round_up(D.Rk, kPadRows);
  D.Cp = (int)round_up(D.Ck, kPadCols);
  D.Urp = (int)round_up(D.Ur, kPadRows);
  const bool split_mode = is_split(p);
  const int terms = split_terms_of(p->precision);
  // K chunks of the 16-bit products keep at least a quarter of K: their
  // stages are short, so the chunks' fixed cost and the partials' traffic
  // outweigh a shorter last round (1152 x 1920 pupil, 1000 foci: 4 chunks
  // per tail tile beat 9 by 1.8% per pass; float32, whose stages take ~2.7x
  // longer, is fastest at 9).
  const int chunk_div = split_mode ? 4 : 0;
  p->sched_fwd = make_sched(D.Urp, D.Cp, D.Rp,
                            choose_tile(D.Urp, D.Cp, split_mode, terms, p->cus), p->cus,
                            split_enabled(), chunk_div);
  p->sched_bwd = make_sched(D.Rp, D.Cp, D.Urp,
                            choose_tile(D.Rp, D.Cp, split_mode, terms, p->cus), p->cus,
                            split_enabled(), chunk_div);
  // The two-term split forward product with the fused focus gather on the
  // 16x16-block loop (64 x 128 tiles) when those tiles make one round over
  // at least half of the CUs (1152 x 1920, 1000 foci: 240 tiles; 2.7% faster
  // per pass than the 32x32-block direct loop on the same tiles).
  // GSWMTP_FWD_LOOP=d16|default forces either (d16 up to one round).
  if (split_mode && terms == 2 && D.Urp % 64 == 0 && D.Cp % 128 == 0) {
    const long t16 = (long)(D.Urp / 64) * (D.Cp / 128);
    bool d16 = t16 <= p->cus && 2 * t16 >= p->cus;
    if (const char *fl = std::getenv("GSWMTP_FWD_LOOP")) {
      if (std::strcmp(fl, "d16") == 0) d16 = t16 <= p->cus;
      if (std::strcmp(fl, "default") == 0) d16 = false;
    }
    if (d16) {
      p->sched_fwd = make_sched(D.Urp, D.Cp, D.Rp, GemmTile{64, 128, 32, 1, 3}, p->cus, false);
      const char *gm = std::getenv("GSWMTP_XCD_GM");
      p->sched_fwd.xgm = gm ? std::max(1, std::atoi(gm)) : 2;
      if (p->sched_fwd.tiles_m % p->sched_fwd.xgm) p->sched_fwd.xgm = 1;
    }
  }
  // Two-term split adjoint on 48 x 192 tiles (the 16x16-block loop) when its
  // default tiles would need a split-K second round and the 48 x 192 tiles
  // make one round over at least 85% of the CUs (1152 x 1920: 240 tiles
  // against 540 of 64 x 64).  GSWMTP_ADJ_LOOP=d16|default forces either
  // (d16 where the shape allows); GSWMTP_XCD_GM=g sets its XCD groups along M.
  if (split_mode && terms == 2 && D.Rp % 48 == 0 && D.Cp % 192 == 0) {
    const long t16 = (long)(D.Rp / 48) * (D.Cp / 192);
    bool d16 = p->sched_bwd.n_tail > 0 && t16 <= p->cus && 100 * t16 >= 85L * p->cus;
    if (const char *al = std::getenv("GSWMTP_ADJ_LOOP")) {
      if (std::strcmp(al, "d16") == 0) d16 = true;
      if (std::strcmp(al, "default") == 0) d16 = false;
    }
    if (d16) {
      p->sched_bwd = make_sched(D.Rp, D.Cp, D.Urp, GemmTile{48, 192, 32, 1, 3}, p->cus, false);
      const char *gm = std::getenv("GSWMTP_XCD_GM");
      p->sched_bwd.xgm = gm ? std::max(1, std::atoi(gm)) : 2;
      if (p->sched_bwd.tiles_m % p->sched_bwd.xgm) p->sched_bwd.xgm = 1;
    }
  }
  // Grid form (float32): when the foci fill a quarter or more of the reduced
  // grid and are many enough to repay its extra launches (measured
  // crossover: the per-focus gather and scatter cost ~0.09 us per focus and
  // pass, the grid form ~0.02 us plus ~20 us of launches, even at about 370
  // foci), the second product of Eq. 2 is formed densely on the matrix cores
  // (as the paper does) instead of per focus.  GSWMTP_SECOND=gather|grid
  // forces either form.
  p->grid_form = (double)D.Ur * D.Uc <= 4.0 * D.nf && D.nf >= 384;
  if (const char *sf = std::getenv("GSWMTP_SECOND")) {
    if (std::strcmp(sf, "gather") == 0) p->grid_form = false;
    if (std::strcmp(sf, "grid") == 0) p->grid_form = true;
  }
  D.Ucp = (int)round_up(D.Uc, kPadCols);
  // Split modes with one focus in every reduced row (N = U_r, e.g. random
  // foci): the adjoint takes Omega_r^H diag(Theta') as its left operand and
  // the conjugated Omega_c rows of the foci, fixed at plan time, as its
  // right one, in place of the per-pass scatter into S.
  // GSWMTP_ADJOINT=scatter keeps the scatter.
  p->scaled_adj = split_mode && !p->grid_form && D.nf == D.Ur;
  if (const char *sa = std::getenv("GSWMTP_ADJOINT"))
    if (std::strcmp(sa, "scatter") == 0) p->scaled_adj = false;
  if (p->grid_form) {
    // the first product L^T = P^T Omega_r^T in the plan's precision; the grid
    // product and the grid scatter's product in float32 (small: U_r x U_c)
    p->sched_f1 = make_sched(D.Cp, D.Urp, D.Rp,
                             choose_tile(D.Cp, D.Urp, split_mode, terms, p->cus), p->cus,
                             split_enabled(), chunk_div);
    if (p->sched_f1.tile.pipe == 2) p->sched_f1.tile.pipe = 1;   // the pipelined loop
    p->sched_f2 = make_sched(D.Urp, D.Ucp, D.Cp, choose_tile(D.Urp, D.Ucp, false), p->cus,
                             split_enabled());
    p->sched_a1 = make_sched(D.Urp, D.Cp, D.Ucp, choose_tile(D.Urp, D.Cp, false), p->cus,
                             split_enabled());
  }

}

// Split-K partials of the plan's products (floats, at least 1).
size_t part_floats_of(const gswmtp_plan *p) {
  size_t f = std::max<size_t>(std::max(p->sched_fwd.part_floats, p->sched_bwd.part_floats), 1);
  if (p->grid_form)
    f = std::max({f, p->sched_f1.part_floats, p->sched_f2.part_floats, p->sched_a1.part_floats});
  return f;
}

// Pool 1 (kernel matrices, pupil and product buffers), after derive_layout.
void carve_pool1(Carver &c, Bufs &b, const gswmtp_plan *p) {
  const Dims &D = p->d;
  const size_t nf = D.nf;
  const size_t Rp = D.Rp, Cp = D.Cp, Urp = D.Urp, Uc = D.Uc, Ucp = D.Ucp;
  const size_t Ucr = p->grid_form ? Ucp : Uc;   // Omega_c rows (zero-padded in the grid form)
  const bool split = is_split(p);
  const size_t nt = (size_t)split_terms_of(p->precision);
  const size_t f32 = split ? 0 : 1;       // float32-only buffers
  const size_t part_floats = part_floats_of(p);
  b.omt_r = c.take<float>(f32 * Rp * Urp); b.omt_i = c.take<float>(f32 * Rp * Urp);
  b.omc_r = c.take<float>(f32 * Rp * Urp); b.omc_i = c.take<float>(f32 * Rp * Urp);
  b.wc_r = c.take<float>(Ucr * Cp); b.wc_i = c.take<float>(Ucr * Cp);
  b.amp = c.take<float>(Rp * Cp);
  b.p_r = c.take<float>(f32 * Rp * Cp); b.p_i = c.take<float>(f32 * Rp * Cp);
  // gather partials: one per forward column tile and focus, sized for the
  // narrowest tile (64 columns) so that a batch may run any tile width
  b.gpart = c.take<float>(2 * (size_t)(Cp / 64) * ((nf + 1) & ~(size_t)1));
  const size_t fs = f32 || p->grid_form ? 1 : 0;   // float32 S (split grid form too)
  b.s_r = c.take<float>(fs * Urp * Cp); b.s_i = c.take<float>(fs * Urp * Cp);
  b.x_r = c.take<float>(Rp * Cp); b.x_i = c.take<float>(Rp * Cp);
  b.part = c.take<float>(part_floats);
  b.as_f = c.take<unsigned short>(2 * nt * Urp * Rp);
  b.as_b = c.take<unsigned short>(2 * nt * Rp * Urp);
  b.ps = c.take<unsigned short>(2 * nt * Cp * Rp);
  b.xs = c.take<unsigned short>(2 * nt * Cp * Rp);
  b.ss = c.take<unsigned short>(2 * nt * Cp * Urp);
  const size_t sa = p->scaled_adj ? 1 : 0;
  b.ob_r = c.take<float>(sa * Rp * Urp); b.ob_i = c.take<float>(sa * Rp * Urp);
  b.as_s = c.take<unsigned short>(sa * 2 * nt * Rp * Urp);
  b.bs = c.take<unsigned short>(sa * 2 * nt * Cp * Urp);
  b.unit = c.take<float>(sa * 2 * nf);
  const size_t gf = p->grid_form ? 1 : 0;
  b.lt_r = c.take<float>(gf * Cp * Urp); b.lt_i = c.take<float>(gf * Cp * Urp);
  b.wt_r = c.take<float>(gf * Cp * Ucp); b.wt_i = c.take<float>(gf * Cp * Ucp);
  b.wn_i = c.take<float>(gf * Ucp * Cp);
  b.g_r = c.take<float>(gf * Urp * Ucp); b.g_i = c.take<float>(gf * Urp * Ucp);
  b.tg_r = c.take<float>(gf * Ucp * Urp); b.tg_i = c.take<float>(gf * Ucp * Urp);
}

int plan_build(gswmtp_plan *p, const gswmtp_desc *d) {
  Dims &D = p->d;
  D.ny = d->ny;
  D.nx = d->nx;
  D.nf = d->n_foci;
  p->precision = d->precision;
  p->weighting = d->weighting;
  // float16 terms need operands near unit scale: the pupil carries
  // A * 2^amp_exp with max A * 2^amp_exp in [0.5, 1); the gather undoes it.
  if (p->precision == GSWMTP_FP16X3) {
    double amax = 1.0;
    if (d->amplitude) {
      amax = 0.0;
      for (size_t i = 0; i < (size_t)d->ny * d->nx; ++i)
        amax = std::max(amax, (double)d->amplitude[i]);
    }
    p->amp_exp = scale_exponent(amax);
  }
  const char *ng = std::getenv("GSWMTP_NO_GRAPH");
  p->use_graph = !(ng && std::atoi(ng) != 0);

  const size_t nf = D.nf, ny = D.ny, nx = D.nx, np = ny * nx;
  HIP_TRY(p, hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
  HIP_TRY(p, hipEventCreateWithFlags(&p->ev_user, hipEventDisableTiming));
  HIP_TRY(p, hipEventCreateWithFlags(&p->ev_int, hipEventDisableTiming));
  HIP_TRY(p, enter(p));
  hipStream_t s = p->stream;

  // ---- pool 0: inputs, index work, per-focus state ----

  {
    Carver c(nullptr);
    carve_pool0(c, p->b, nf, ny, nx);
    p->pool0_bytes = c.off;
  }
  if (p->ws) {
    if (p->pool0_bytes > p->ws_bytes)
      return fail(p, GSWMTP_E_NOMEM, "workspace smaller than the index pool");
    p->pool0 = p->ws;
  } else if (fault_alloc_hit(p->fault_alloc, &p->n_alloc)) {
    return fail(p, GSWMTP_E_NOMEM, "device allocation (index pool): injected failure");
  } else if (hipMalloc(&p->pool0, p->pool0_bytes) != hipSuccess) {
    return fail(p, GSWMTP_E_NOMEM, "device allocation (index pool)");
  }
  {
    Carver c(p->pool0);
    carve_pool0(c, p->b, nf, ny, nx);
  }
  Bufs &b = p->b;
  HIP_TRY(p, hipMemsetAsync(p->pool0, 0, p->pool0_bytes, s));

  // ---- inputs ----
  std::vector<double> uc(nx), vc(ny);
  for (size_t i = 0; i < nx; ++i) uc[i] = d->u ? d->u[i] : (double)i - (double)(nx - 1) / 2.0;
  for (size_t j = 0; j < ny; ++j) vc[j] = d->v ? d->v[j] : (double)j - (double)(ny - 1) / 2.0;
  HIP_TRY(p, hipMemcpyAsync(b.fx, d->fx, nf * 8, hipMemcpyHostToDevice, s));
  if (d->fz)
    HIP_TRY(p, hipMemcpyAsync(b.fz, d->fz, nf * 8, hipMemcpyHostToDevice, s));
  else
    hipLaunchKernelGGL(k_fill_d, grid1(nf), dim3(256), 0, s, b.fz, 0.0, nf);
  HIP_TRY(p, hipMemcpyAsync(b.fy, d->fy, nf * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(p, hipMemcpyAsync(b.target, d->target, nf * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(p, hipMemcpyAsync(b.ucoord, uc.data(), nx * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(p, hipMemcpyAsync(b.vcoord, vc.data(), ny * 8, hipMemcpyHostToDevice, s));
  if (d->amplitude) {
    HIP_TRY(p, hipMemcpyAsync(b.aeff, d->amplitude, np * 4, hipMemcpyHostToDevice, s));
  } else {
    hipLaunchKernelGGL(k_fill_f, grid1(np), dim3(256), 0, s, b.aeff, 1.f, np);
  }
  if (d->mask) {
    auto *m = reinterpret_cast<unsigned char *>(b.iobuf);
    HIP_TRY(p, hipMemcpyAsync(m, d->mask, np, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_aeff, grid1(np), dim3(256), 0, s, b.aeff, m, np);
  }

  // ---- index work ----
  int *sc = b.scalars;  // 0 ux, 1 uy, 2 ny_kept, 3 nx_kept, 4 n_ap
  hipLaunchKernelGGL(k_keep, dim3((unsigned)ny), dim3(256), 0, s, b.aeff, (int)ny, (int)nx,
                     (size_t)nx, (size_t)1, b.keep_row);
  hipLaunchKernelGGL(k_keep, dim3((unsigned)nx), dim3(256), 0, s, b.aeff, (int)nx, (int)ny,
                     (size_t)1, (size_t)nx, b.keep_col);
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, b.keep_row, (int)ny, b.rows,
                     b.row_pos, sc + 2);
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, b.keep_col, (int)nx, b.cols,
                     b.col_pos, sc + 3);
  hipLaunchKernelGGL(k_aperture_part, dim3(kApBlocks), dim3(256), 0, s, b.aeff, np, b.ap_part,
                     b.ap_cnt);
  hipLaunchKernelGGL(k_aperture_sum, dim3(1), dim3(kApBlocks), 0, s, b.ap_part, b.ap_cnt, sc + 4,
                     b.dscalars);
  const dim3 gf = grid1(nf);
  IndexScratch isc{{b.skey0, b.skey1}, {b.sval0, b.sval1}, b.shist, b.shead, b.srank};
  const bool has_z = d->fz != nullptr;
  HIP_TRY(p, unique_pairs(b.fx, b.fz, has_z, (int)nf, isc, b.ix, b.xu, b.xzu, sc + 0, s));
  HIP_TRY(p, unique_pairs(b.fy, b.fz, has_z, (int)nf, isc, b.iy, b.yu, b.yzu, sc + 1, s));
  // duplicates, and the focus order of the compressed rows when y is the
  // row axis (the x-row order is sorted again once the axis is known)
  HIP_TRY(p, pair_order(b.iy, b.ix, (int)nf, isc, b.csr_foci, b.dup, s));
  hipLaunchKernelGGL(k_tnorm, dim3(1), dim3(1024), 0, s, b.target, (int)nf, b.tnorm, b.tinv,
                     b.tsqrt);
  HIP_TRY(p, hipGetLastError());

  int hs[8] = {0};
  int hdup = 0;
  double hsum = 0.0;
  HIP_TRY(p, hipMemcpyAsync(hs, sc, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(p, hipMemcpyAsync(&hdup, b.dup, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(p, hipMemcpyAsync(&hsum, b.dscalars, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(p, hipStreamSynchronize(s));
  D.ux = hs[0];
  D.uy = hs[1];
  D.ny_kept = hs[2];
  D.nx_kept = hs[3];
  D.n_ap = hs[4];
  D.sum_a2 = hsum;
  if (hdup) return fail(p, GSWMTP_E_DUPFOCUS, "two foci share the same (x, y, z)");
  if (D.n_ap == 0 || D.ny_kept == 0 || D.nx_kept == 0 || !(D.sum_a2 > 0.0))
    return fail(p, GSWMTP_E_EMPTYAPERTURE, "amplitude is zero everywhere");

  // ---- axis, sizes, schedules ----
  derive_layout(p, d);

  // ---- pool 1: kernel matrices, pupil and product buffers ----
  const size_t Rp = D.Rp, Cp = D.Cp, Urp = D.Urp, Uc = D.Uc, Ucp = D.Ucp;
  const bool split = is_split(p);
  {
    Carver c(nullptr);
    carve_pool1(c, p->b, p);
    p->pool1_bytes = c.off;
  }
  if (p->ws) {
    const size_t off = round_up(p->pool0_bytes, 256);
    if (off + p->pool1_bytes > p->ws_bytes) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "workspace too small: %zu bytes needed",
                    off + p->pool1_bytes);
      return fail(p, GSWMTP_E_NOMEM, msg);
    }
    p->pool1 = static_cast<char *>(p->ws) + off;
  } else if (fault_alloc_hit(p->fault_alloc, &p->n_alloc)) {
    return fail(p, GSWMTP_E_NOMEM, "device allocation (product pool): injected failure");
  } else if (hipMalloc(&p->pool1, p->pool1_bytes) != hipSuccess) {
    return fail(p, GSWMTP_E_NOMEM, "device allocation (product pool)");
  }
  {
    Carver c(p->pool1);
    carve_pool1(c, p->b, p);
  }
  HIP_TRY(p, hipMemsetAsync(p->pool1, 0, p->pool1_bytes, s));

  const int *ir = D.axis == 0 ? b.iy : b.ix;
  const int *ic = D.axis == 0 ? b.ix : b.iy;
  if (D.axis != 0) HIP_TRY(p, pair_order(ir, ic, (int)nf, isc, b.csr_foci, nullptr, s));
  hipLaunchKernelGGL(k_row_ptr, grid1(nf + 1), dim3(256), 0, s, ir, b.csr_foci, (int)nf, D.Ur,
                     b.csr_ptr);
  hipLaunchKernelGGL(k_csr_gather, grid1(nf), dim3(256), 0, s, ic, b.csr_foci, (int)nf, b.csr_ic);
  hipLaunchKernelGGL(k_csr_gather, grid1(nf), dim3(256), 0, s, ir, b.csr_foci, (int)nf, b.csr_ir);
  const double *rcoord = D.axis == 0 ? b.vcoord : b.ucoord;
  const double *ccoord = D.axis == 0 ? b.ucoord : b.vcoord;
  const int *rkept = D.axis == 0 ? b.rows : b.cols;
  const int *ckept = D.axis == 0 ? b.cols : b.rows;
  const double *rfu = D.axis == 0 ? b.yu : b.xu;
  const double *cfu = D.axis == 0 ? b.xu : b.yu;
  const double *rfz = D.axis == 0 ? b.yzu : b.xzu;
  const double *cfz = D.axis == 0 ? b.xzu : b.yzu;
  const double s_r = D.axis == 0 ? d->s_y : d->s_x;
  const double s_c = D.axis == 0 ? d->s_x : d->s_y;
  if (split) {
#define OMEGA(BF, NT)                                                                          \
  hipLaunchKernelGGL((k_omega_r_split<BF, NT>), grid1(Rp * Urp), dim3(256), 0, s, rcoord, rkept, \
                     D.Rk, rfu, rfz, D.Ur, s_r, D.Rp, D.Urp, b.as_f, b.as_b,             \
                     p->scaled_adj ? b.ob_r : nullptr, p->scaled_adj ? b.ob_i : nullptr)
    DISPATCH_SPLIT(p->precision, OMEGA)
#undef OMEGA
  } else {
    hipLaunchKernelGGL(k_omega_r, grid1(Rp * Urp), dim3(256), 0, s, rcoord, rkept, D.Rk, rfu,
                       rfz, D.Ur, s_r, D.Rp, D.Urp, b.omt_r, b.omt_i, b.omc_r, b.omc_i);
  }
  hipLaunchKernelGGL(k_omega_c, grid1(Uc * Cp), dim3(256), 0, s, ccoord, ckept, D.Ck, cfu, cfz,
                     D.Uc, s_c, D.Cp, b.wc_r, b.wc_i);
  if (p->scaled_adj) {   // right operand of the scaled adjoint: S^T for unit Theta'
    hipLaunchKernelGGL(k_fill_unit, grid1(nf), dim3(256), 0, s, b.unit, (int)nf);
    HIP_TRY(p, launch_scatter_split(p, b.unit, 1.f, false, s, b.bs));
  }
  if (p->grid_form)
    hipLaunchKernelGGL(k_grid_tables, grid1(Ucp * Cp), dim3(256), 0, s, b.wc_r, b.wc_i, D.Uc,
                       D.Cp, D.Ucp, b.wt_r, b.wt_i, b.wn_i);
  const Orient o = orient_of(p);
  hipLaunchKernelGGL(k_encode_amp, grid1(Rp * Cp), dim3(256), 0, s, o, b.aeff,
                     std::ldexp(1.f, p->amp_exp), (int)nx, D.Rp, D.Cp, b.amp);
  const float *phi_dev = nullptr;
  if (d->phi0) {
    HIP_TRY(p, hipMemcpyAsync(b.iobuf, d->phi0, np * 4, hipMemcpyHostToDevice, s));
    phi_dev = b.iobuf;
  }
  HIP_TRY(p, encode_phase(p, phi_dev, s, false));
  hipLaunchKernelGGL(k_fill_d, grid1(nf), dim3(256), 0, s, b.w, 1.0, nf);
  HIP_TRY(p, hipGetLastError());
  HIP_TRY(p, hipStreamSynchronize(s));
  HIP_TRY(p, leave(p));
  return GSWMTP_OK;
}

thread_local std::string g_last_create_error;

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

// ---------------------------------------------------------------------------
// Scratch of the allocation-free operator call: one array per device
// ---------------------------------------------------------------------------

// 64 MiB covers the forward operator's scratch up to ~2.9 M pupil samples
// (float32 or two-term split), e.g. 1152 x 1920 with 1000 foci (~36 MB).
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per
// device, with that device current; host code never passes the array's name).
hipError_t static_scratch_of(int device, char **out) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<char *>(ptr);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}
}  // namespace

extern "C" {

int gswmtp_version(void) { return GSWMTP_VERSION; }

const char *gswmtp_status_string(int status) {
  switch (status) {
    case GSWMTP_OK: return "GSWMTP_OK";
    case GSWMTP_E_INVAL: return "GSWMTP_E_INVAL: invalid argument";
    case GSWMTP_E_DUPFOCUS: return "GSWMTP_E_DUPFOCUS: duplicate focus";
    case GSWMTP_E_EMPTYAPERTURE: return "GSWMTP_E_EMPTYAPERTURE: empty aperture";
    case GSWMTP_E_NOMEM: return "GSWMTP_E_NOMEM: out of memory";
    case GSWMTP_E_HIP: return "GSWMTP_E_HIP: HIP runtime error";
    case GSWMTP_E_NONFINITE: return "GSWMTP_E_NONFINITE: non-finite focus intensities";
    case GSWMTP_E_NODEV: return "GSWMTP_E_NODEV: no gfx950 device";
    case GSWMTP_E_UNSUPPORTED: return "GSWMTP_E_UNSUPPORTED: not supported";
  }
  return "unknown status";
}

const char *gswmtp_last_error(const gswmtp_plan *p) {
  if (!p) return g_last_create_error.c_str();
  return p->err.c_str();
}

int gswmtp_desc_init(gswmtp_desc *d) {
  if (!d) return GSWMTP_E_INVAL;
  std::memset(d, 0, sizeof *d);
  d->precision = GSWMTP_FP32;
  d->axis = -1;
  d->weighting = GSWMTP_WEIGHT_GSW;
  return GSWMTP_OK;
}

static int create_impl(gswmtp_plan **out, const gswmtp_desc *d, void *ws, size_t ws_bytes,
                       void *stream);

// Distinct canonical (coordinate, z) keys of one axis, counted on the host
// (sizing only; the plan's own index work runs on the device).
static int count_keys(const double *c, const double *z, size_t n) {
  std::vector<std::pair<double, double>> k(n);
  for (size_t i = 0; i < n; ++i) {
    const double a = c[i] == 0.0 ? 0.0 : c[i];
    const double b = z ? (z[i] == 0.0 ? 0.0 : z[i]) : 0.0;
    k[i] = {a, b};
  }
  std::sort(k.begin(), k.end());
  return (int)(std::unique(k.begin(), k.end()) - k.begin());
}

int gswmtp_plan_workspace_size(const gswmtp_desc *d, size_t *bytes) {
  if (!bytes) return GSWMTP_E_INVAL;
  *bytes = 0;
  const int v = validate(d);
  if (v != GSWMTP_OK) return v;
  gswmtp_plan t;
  try {
    Dims &D = t.d;
    D.ny = d->ny;
    D.nx = d->nx;
    D.nf = d->n_foci;
    D.ux = count_keys(d->fx, d->fz, D.nf);
    D.uy = count_keys(d->fy, d->fz, D.nf);
    std::vector<char> keep_r(d->ny, 0), keep_c(d->nx, 0);
    for (int y = 0; y < d->ny; ++y)
      for (int x = 0; x < d->nx; ++x) {
        const size_t i = (size_t)y * d->nx + x;
        const float a = d->mask && !d->mask[i] ? 0.f : d->amplitude ? d->amplitude[i] : 1.f;
        if (a > 0.f) keep_r[y] = keep_c[x] = 1;
      }
    D.ny_kept = (int)std::count(keep_r.begin(), keep_r.end(), 1);
    D.nx_kept = (int)std::count(keep_c.begin(), keep_c.end(), 1);
  } catch (const std::bad_alloc &) {
    return GSWMTP_E_NOMEM;
  }
  if (t.d.ny_kept == 0 || t.d.nx_kept == 0) return GSWMTP_E_EMPTYAPERTURE;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      cus > 0)
    t.cus = cus;
  else
    t.cus = 256;
  t.precision = d->precision;
  derive_layout(&t, d);
  Carver c0(nullptr), c1(nullptr);
  carve_pool0(c0, t.b, t.d.nf, t.d.ny, t.d.nx);
  carve_pool1(c1, t.b, &t);
  *bytes = round_up(c0.off, 256) + c1.off;
  return GSWMTP_OK;
}

int gswmtp_plan_create_with_workspace(gswmtp_plan **out, const gswmtp_desc *d, void *dev_ws,
                                      size_t bytes, void *stream) {
  if (!out) return GSWMTP_E_INVAL;
  *out = nullptr;
  g_last_create_error.clear();
  if (!dev_ws || bytes == 0 || reinterpret_cast<uintptr_t>(dev_ws) % 256 != 0) {
    g_last_create_error = "workspace must be non-null, non-empty and 256-byte aligned";
    return GSWMTP_E_INVAL;
  }
  return create_impl(out, d, dev_ws, bytes, stream);
}

int gswmtp_plan_create(gswmtp_plan **out, const gswmtp_desc *d, void *stream) {
  if (!out) return GSWMTP_E_INVAL;
  *out = nullptr;
  g_last_create_error.clear();
  return create_impl(out, d, nullptr, 0, stream);
}

static int create_impl(gswmtp_plan **out, const gswmtp_desc *d, void *ws, size_t ws_bytes,
                       void *stream) {
  const int v = validate(d);
  if (v != GSWMTP_OK) {
    g_last_create_error = "invalid plan descriptor";
    return v;
  }
  gswmtp_plan *p = new (std::nothrow) gswmtp_plan();
  if (!p) return GSWMTP_E_NOMEM;
  p->ws = ws;
  p->ws_bytes = ws_bytes;
  p->user_stream = static_cast<hipStream_t>(stream);
  p->fault_alloc = ws ? -1 : fault_alloc_setting();   // a caller's workspace: no allocation
  if (p->fault_alloc == 0) {
    g_last_create_error = "device allocation: injected failure (GSWMTP_FAULT_INJECT=alloc)";
    delete p;
    return GSWMTP_E_NOMEM;
  }
  int rc = check_device(p);
  if (rc == GSWMTP_OK) {
    try {
      rc = plan_build(p, d);
    } catch (const std::bad_alloc &) {
      rc = fail(p, GSWMTP_E_NOMEM, "host allocation");
    }
  }
  if (rc != GSWMTP_OK) {
    g_last_create_error = p->err;
    free_plan(p);
    return rc;
  }
  *out = p;
  return GSWMTP_OK;
}

int gswmtp_plan_destroy(gswmtp_plan *p) {
  if (!p) return GSWMTP_OK;
  DeviceGuard g(p->device);
  free_plan(p);
  return GSWMTP_OK;
}

int gswmtp_set_stream(gswmtp_plan *p, void *stream) {
  if (!p) return GSWMTP_E_INVAL;
  p->user_stream = static_cast<hipStream_t>(stream);
  return GSWMTP_OK;
}

int gswmtp_sync(gswmtp_plan *p) {
  if (!p) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  return GSWMTP_OK;
}

int gswmtp_iterate(gswmtp_plan *p, int n_iter, double stop_accuracy) {
  if (!p || n_iter < 0 || !std::isfinite(stop_accuracy)) return GSWMTP_E_INVAL;
  if (n_iter == 0) return GSWMTP_OK;
  DeviceGuard g(p->device);
  HIP_TRY(p, enter(p));
  hipLaunchKernelGGL(k_control, dim3(1), dim3(1), 0, p->stream, p->b.ctrl, p->b.stats,
                     stop_accuracy);
  HIP_TRY(p, hipGetLastError());
  if (p->use_graph) {
    if (!p->graph1) HIP_TRY(p, capture(p, 1, &p->graph1));
    if (n_iter >= 8 && !p->graph8) HIP_TRY(p, capture(p, 8, &p->graph8));
    int left = n_iter;
    for (; left >= 8; left -= 8) HIP_TRY(p, hipGraphLaunch(p->graph8, p->stream));
    for (; left > 0; --left) HIP_TRY(p, hipGraphLaunch(p->graph1, p->stream));
  } else {
    for (int i = 0; i < n_iter; ++i) HIP_TRY(p, enqueue_pass(p, p->stream));
  }
  p->fwd_valid = p->stats_valid = false;
  HIP_TRY(p, leave(p));
  return GSWMTP_OK;
}

int gswmtp_iterate_measured(gswmtp_plan *p, const double *measured) {
  if (!p || !measured) return GSWMTP_E_INVAL;
  const size_t nf = (size_t)p->d.nf;
  double sum = 0.0;
  for (size_t n = 0; n < nf; ++n) {
    if (!std::isfinite(measured[n]) || measured[n] < 0.0)
      return fail(p, GSWMTP_E_INVAL, "measured intensities must be finite and >= 0");
    sum += measured[n];
  }
  if (!(sum > 0.0) || !std::isfinite(sum))
    return fail(p, GSWMTP_E_INVAL, "measured intensities must have a finite positive sum");
  DeviceGuard g(p->device);
  HIP_TRY(p, enter(p));
  HIP_TRY(p, hipMemcpyAsync(p->b.meas, measured, 8 * nf, hipMemcpyHostToDevice, p->stream));
  hipLaunchKernelGGL(k_meas_norm, dim3(1), dim3(1024), 0, p->stream, p->b.meas, (int)nf);
  hipLaunchKernelGGL(k_control, dim3(1), dim3(1), 0, p->stream, p->b.ctrl, p->b.stats, 0.0);
  HIP_TRY(p, hipGetLastError());
  p->meas_active = p->b.meas;
  const hipError_t e = enqueue_pass(p, p->stream);   // eager: graphs hold no measured pass
  p->meas_active = nullptr;
  HIP_TRY(p, e);
  p->fwd_valid = p->stats_valid = false;
  HIP_TRY(p, leave(p));
  HIP_TRY(p, hipStreamSynchronize(p->stream));        // the caller may reuse `measured`
  return GSWMTP_OK;
}

int gswmtp_iterations_done(gswmtp_plan *p, int *n) {
  if (!p || !n) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  int c[CTRL_N];
  HIP_TRY(p, enter(p));
  HIP_TRY(p, hipMemcpyAsync(c, p->b.ctrl, sizeof c, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  *n = c[CTRL_ITERS];
  if (c[CTRL_NONFINITE]) return fail(p, GSWMTP_E_NONFINITE, "focus intensities became non-finite");
  return GSWMTP_OK;
}

int gswmtp_get_phase_device(gswmtp_plan *p, float *dev_out) {
  if (!p || !dev_out) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  HIP_TRY(p, enter(p));
  HIP_TRY(p, phase_out(p, dev_out, p->stream));
  HIP_TRY(p, leave(p));
  return GSWMTP_OK;
}

int gswmtp_get_phase(gswmtp_plan *p, float *out) {
  if (!p || !out) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  const size_t np = (size_t)p->d.ny * p->d.nx;
  HIP_TRY(p, enter(p));
  HIP_TRY(p, phase_out(p, p->b.iobuf, p->stream));
  HIP_TRY(p, hipMemcpyAsync(out, p->b.iobuf, np * 4, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  return GSWMTP_OK;
}

static int set_phase_impl(gswmtp_plan *p, const float *dev_phi) {
  HIP_TRY(p, encode_phase(p, dev_phi, p->stream, true));
  p->fwd_valid = p->stats_valid = false;
  return GSWMTP_OK;
}

int gswmtp_set_phase(gswmtp_plan *p, const float *phi) {
  if (!p || !phi) return GSWMTP_E_INVAL;
  const size_t np = (size_t)p->d.ny * p->d.nx;
  if (!finite_all(phi, np)) return fail(p, GSWMTP_E_INVAL, "non-finite phase");
  DeviceGuard g(p->device);
  HIP_TRY(p, enter(p));
  HIP_TRY(p, hipMemcpyAsync(p->b.iobuf, phi, np * 4, hipMemcpyHostToDevice, p->stream));
  int rc = set_phase_impl(p, p->b.iobuf);
  if (rc) return rc;
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  return GSWMTP_OK;
}

int gswmtp_set_phase_device(gswmtp_plan *p, const float *dev_phi) {
  if (!p || !dev_phi) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  HIP_TRY(p, enter(p));
  int rc = set_phase_impl(p, dev_phi);
  if (rc) return rc;
  HIP_TRY(p, leave(p));
  return GSWMTP_OK;
}

int gswmtp_get_foci_field_device(gswmtp_plan *p, float *dev_field, float *dev_intensity) {
  if (!p || (!dev_field && !dev_intensity)) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  HIP_TRY(p, enter(p));
  if (!p->fwd_valid) {   // the forward's field kernel writes the caller's buffers too
    HIP_TRY(p, stage_forward(p, false, p->stream, false));
    HIP_TRY(p, launch_field(p, p->stream, dev_field, dev_intensity));
    p->fwd_valid = true;
  } else {
    const size_t nf = p->d.nf;
    if (dev_field)
      HIP_TRY(p, hipMemcpyAsync(dev_field, p->b.theta, 8 * nf, hipMemcpyDeviceToDevice,
                                p->stream));
    if (dev_intensity)
      HIP_TRY(p, hipMemcpyAsync(dev_intensity, p->b.intensity, 4 * nf, hipMemcpyDeviceToDevice,
                                p->stream));
  }
  HIP_TRY(p, leave(p));
  return GSWMTP_OK;
}

int gswmtp_get_foci_field(gswmtp_plan *p, float *out) {
  if (!p || !out) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  HIP_TRY(p, enter(p));
  HIP_TRY(p, ensure_forward(p, false));
  HIP_TRY(p, hipMemcpyAsync(out, p->b.theta, 8 * (size_t)p->d.nf, hipMemcpyDeviceToHost,
                            p->stream));
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  return GSWMTP_OK;
}

int gswmtp_get_stats(gswmtp_plan *p, double *xi, double *eta, double *uniformity) {
  if (!p) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  HIP_TRY(p, enter(p));
  HIP_TRY(p, ensure_forward(p, true));
  double st[ST_N];
  HIP_TRY(p, hipMemcpyAsync(st, p->b.stats, sizeof st, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  if (xi) *xi = st[ST_XI];
  if (eta) *eta = st[ST_ETA];
  if (uniformity) *uniformity = st[ST_U];
  return GSWMTP_OK;
}

int gswmtp_get_weights(gswmtp_plan *p, double *out) {
  if (!p || !out) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  HIP_TRY(p, enter(p));
  HIP_TRY(p, hipMemcpyAsync(out, p->b.w, 8 * (size_t)p->d.nf, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  return GSWMTP_OK;
}

int gswmtp_set_weights(gswmtp_plan *p, const double *w) {
  if (!p || !w) return GSWMTP_E_INVAL;
  if (!finite_all(w, (size_t)p->d.nf)) return fail(p, GSWMTP_E_INVAL, "non-finite weights");
  DeviceGuard g(p->device);
  HIP_TRY(p, enter(p));
  HIP_TRY(p, hipMemcpyAsync(p->b.w, w, 8 * (size_t)p->d.nf, hipMemcpyHostToDevice, p->stream));
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  return GSWMTP_OK;
}

int gswmtp_get_history(gswmtp_plan *p, double *buf, int cap, int *n) {
  if (!p || !n || cap < 0 || (cap > 0 && !buf)) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  int c[CTRL_N];
  HIP_TRY(p, enter(p));
  HIP_TRY(p, hipMemcpyAsync(c, p->b.ctrl, sizeof c, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  const int total = c[CTRL_HIST];
  const int stored = total < kHistCap ? total : kHistCap;
  const int take = stored < cap ? stored : cap;
  std::vector<double> h(3 * (size_t)kHistCap);
  if (take > 0) {
    HIP_TRY(p, hipMemcpy(h.data(), p->b.hist, h.size() * 8, hipMemcpyDeviceToHost));
    for (int k = 0; k < take; ++k) {
      const int idx = (total - take + k) % kHistCap;
      for (int q = 0; q < 3; ++q) buf[3 * k + q] = h[3 * (size_t)idx + q];
    }
  }
  *n = take;
  return GSWMTP_OK;
}

int gswmtp_get_state(gswmtp_plan *p, float *phi, double *w, int *iters) {
  if (!p) return GSWMTP_E_INVAL;
  int rc;
  if (phi && (rc = gswmtp_get_phase(p, phi)) != GSWMTP_OK) return rc;
  if (w && (rc = gswmtp_get_weights(p, w)) != GSWMTP_OK) return rc;
  if (iters && (rc = gswmtp_iterations_done(p, iters)) != GSWMTP_OK) return rc;
  return GSWMTP_OK;
}

int gswmtp_set_state(gswmtp_plan *p, const float *phi, const double *w, int iters) {
  if (!p || iters < 0) return GSWMTP_E_INVAL;
  int rc;
  if (phi && (rc = gswmtp_set_phase(p, phi)) != GSWMTP_OK) return rc;
  if (w && (rc = gswmtp_set_weights(p, w)) != GSWMTP_OK) return rc;
  DeviceGuard g(p->device);
  HIP_TRY(p, enter(p));
  hipLaunchKernelGGL(k_set_state, dim3(1), dim3(1), 0, p->stream, p->b.ctrl, iters);
  HIP_TRY(p, hipGetLastError());
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  return GSWMTP_OK;
}

int gswmtp_set_phase_fixing(gswmtp_plan *p, int from_pass) {
  if (!p || from_pass < 0) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  HIP_TRY(p, enter(p));
  hipLaunchKernelGGL(k_set_fix, dim3(1), dim3(1), 0, p->stream, p->b.ctrl, from_pass);
  HIP_TRY(p, hipGetLastError());
  HIP_TRY(p, leave(p));
  return GSWMTP_OK;
}

int gswmtp_get_index(gswmtp_plan *p, gswmtp_index_info *info, int32_t *ix, int32_t *iy,
                     double *xu, double *yu, int32_t *rows, int32_t *cols) {
  if (!p || !info) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  const Dims &D = p->d;
  info->n_foci = D.nf;
  info->ux = D.ux;
  info->uy = D.uy;
  info->ny_kept = D.ny_kept;
  info->nx_kept = D.nx_kept;
  info->axis = D.axis;
  info->n_aperture = D.n_ap;
  info->sum_a2 = D.sum_a2;
  HIP_TRY(p, enter(p));
  HIP_TRY(p, hipStreamSynchronize(p->stream));
  if (ix) HIP_TRY(p, hipMemcpy(ix, p->b.ix, 4 * (size_t)D.nf, hipMemcpyDeviceToHost));
  if (iy) HIP_TRY(p, hipMemcpy(iy, p->b.iy, 4 * (size_t)D.nf, hipMemcpyDeviceToHost));
  if (xu) HIP_TRY(p, hipMemcpy(xu, p->b.xu, 8 * (size_t)D.ux, hipMemcpyDeviceToHost));
  if (yu) HIP_TRY(p, hipMemcpy(yu, p->b.yu, 8 * (size_t)D.uy, hipMemcpyDeviceToHost));
  if (rows) HIP_TRY(p, hipMemcpy(rows, p->b.rows, 4 * (size_t)D.ny_kept, hipMemcpyDeviceToHost));
  if (cols) HIP_TRY(p, hipMemcpy(cols, p->b.cols, 4 * (size_t)D.nx_kept, hipMemcpyDeviceToHost));
  return GSWMTP_OK;
}

static int forward_field_impl(gswmtp_plan *p, const float *E, float *theta);

int gswmtp_forward_field(gswmtp_plan *p, const float *E, float *theta) {
  if (!p || !E || !theta) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  return forward_field_impl(p, E, theta);
}

int gswmtp_forward_field_noalloc(gswmtp_plan *p, const float *E, float *theta) {
  if (!p || !E || !theta) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  char *base = nullptr;
  HIP_TRY(p, static_scratch_of(p->device, &base));
  // the forward call's scratch, carved from the static array in the plan's
  // own sizes; the plan's buffers are put back however the call ends
  const Dims &D = p->d;
  const size_t np = (size_t)D.ny * D.nx, nf = D.nf;
  const size_t Rp = D.Rp, Cp = D.Cp, Urp = D.Urp, Ucp = D.Ucp;
  const size_t nt = (size_t)split_terms_of(p->precision);
  const size_t gf = p->grid_form ? 1 : 0;
  Carver c(base);
  Bufs b = p->b;
  b.iobuf = c.take<float>(2 * np);
  b.x_r = c.take<float>(Rp * Cp); b.x_i = c.take<float>(Rp * Cp);
  b.xs = c.take<unsigned short>(2 * nt * Cp * Rp);
  b.lt_r = c.take<float>(gf * Cp * Urp); b.lt_i = c.take<float>(gf * Cp * Urp);
  b.g_r = c.take<float>(gf * Urp * Ucp); b.g_i = c.take<float>(gf * Urp * Ucp);
  b.gpart = c.take<float>(2 * (size_t)(Cp / 64) * ((nf + 1) & ~(size_t)1));
  b.part = c.take<float>(part_floats_of(p));
  b.theta_new = c.take<float>(2 * nf);
  if (c.off > kStaticScratchBytes) {
    char msg[160];
    snprintf(msg, sizeof msg, "forward_field_noalloc needs %zu bytes of scratch; the static "
             "array holds %zu", c.off, kStaticScratchBytes);
    return fail(p, GSWMTP_E_NOMEM, msg);
  }
  struct Restore {
    gswmtp_plan *p;
    Bufs saved;
    ~Restore() { p->b = saved; }
  } restore{p, p->b};
  // the plan's own scratch starts zeroed at creation: so does this one
  HIP_TRY(p, enter(p));
  hipLaunchKernelGGL(k_fill_f, grid1(c.off / 4), dim3(256), 0, p->stream,
                     reinterpret_cast<float *>(base), 0.f, c.off / 4);
  HIP_TRY(p, hipGetLastError());
  p->b = b;
  return forward_field_impl(p, E, theta);
}

static int forward_field_impl(gswmtp_plan *p, const float *E, float *theta) {
  const Dims &D = p->d;
  const size_t np = (size_t)D.ny * D.nx;
  if (!finite_all(E, 2 * np)) return fail(p, GSWMTP_E_INVAL, "non-finite pupil field");
  HIP_TRY(p, enter(p));
  hipStream_t s = p->stream;
  HIP_TRY(p, hipMemcpyAsync(p->b.iobuf, E, 8 * np, hipMemcpyHostToDevice, s));
  const dim3 gr = grid1((size_t)D.Rp * D.Cp);
  const Orient o = orient_of(p);
  float unscale = 1.f;
  if (is_split(p)) {
    // float16/bfloat16 terms: bring the field to unit scale by a power of two
    double amax = 0.0;
    for (size_t i = 0; i < 2 * np; ++i) amax = std::max(amax, (double)std::fabs(E[i]));
    const int e = p->precision == GSWMTP_FP16X3 ? scale_exponent(amax) : 0;
    const float sc = std::ldexp(1.f, e);
    unscale = std::ldexp(1.f, -e);
#define COMPACT(BF, NT)                                                                     \
  hipLaunchKernelGGL((k_compact_split<BF, NT>), gr, dim3(256), 0, s, o, p->b.iobuf, sc, D.nx, \
                     D.Rp, D.Cp, p->b.xs)
    DISPATCH_SPLIT(p->precision, COMPACT)
#undef COMPACT
    HIP_TRY(p, hipGetLastError());
    if (p->grid_form)
      HIP_TRY(p, split_grid_forward(p, p->b.xs, false, s));
    else
      HIP_TRY(p, launch_cgemm_split(p, true, EPI_GATHER, p->b.xs, nullptr, nullptr, nullptr,
                                    false, s));
  } else {
    hipLaunchKernelGGL(k_compact_complex, gr, dim3(256), 0, s, o, p->b.iobuf, D.nx, D.Rp, D.Cp,
                       p->b.x_r, p->b.x_i);
    HIP_TRY(p, hipGetLastError());
    HIP_TRY(p, forward_products(p, p->b.x_r, p->b.x_i, false, s));
  }
  HIP_TRY(p, launch_gather_reduce(p, p->b.theta_new, unscale, s));
  HIP_TRY(p, hipMemcpyAsync(theta, p->b.theta_new, 8 * (size_t)D.nf, hipMemcpyDeviceToHost, s));
  HIP_TRY(p, hipStreamSynchronize(s));
  return GSWMTP_OK;
}

int gswmtp_adjoint_field(gswmtp_plan *p, const float *theta, float *E) {
  if (!p || !theta || !E) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  const Dims &D = p->d;
  const size_t np = (size_t)D.ny * D.nx;
  if (!finite_all(theta, 2 * (size_t)D.nf)) return fail(p, GSWMTP_E_INVAL, "non-finite field");
  HIP_TRY(p, enter(p));
  hipStream_t s = p->stream;
  HIP_TRY(p, hipMemcpyAsync(p->b.theta_new, theta, 8 * (size_t)D.nf, hipMemcpyHostToDevice, s));
  float unscale = 1.f;
  if (is_split(p)) {
    double amax = 0.0;
    for (size_t i = 0; i < 2 * (size_t)D.nf; ++i)
      amax = std::max(amax, (double)std::fabs(theta[i]));
    const int e = p->precision == GSWMTP_FP16X3 ? scale_exponent(amax) : 0;
    unscale = std::ldexp(1.f, -e);
    if (p->grid_form)
      HIP_TRY(p, split_grid_scatter(p, p->b.theta_new, std::ldexp(1.f, e), false, s));
    else
      HIP_TRY(p, launch_scatter_split(p, p->b.theta_new, std::ldexp(1.f, e), false, s));
    HIP_TRY(p, launch_cgemm_split(p, false, EPI_STORE, p->b.ss, p->b.x_r, p->b.x_i, nullptr,
                                  false, s));
  } else {
    HIP_TRY(p, scatter_products(p, p->b.theta_new, false, s));
    HIP_TRY(p, launch_cgemm(p, false, EPI_STORE, p->b.s_r, p->b.s_i, p->b.x_r, p->b.x_i,
                            nullptr, nullptr, false, s));
  }
  hipLaunchKernelGGL(k_expand_complex, grid1(np), dim3(256), 0, s, p->b.x_r, p->b.x_i,
                     p->b.row_pos, p->b.col_pos, D.axis, D.ny, D.nx, D.Cp, unscale, p->b.iobuf);
  HIP_TRY(p, hipGetLastError());
  HIP_TRY(p, hipMemcpyAsync(E, p->b.iobuf, 8 * np, hipMemcpyDeviceToHost, s));
  HIP_TRY(p, hipStreamSynchronize(s));
  return GSWMTP_OK;
}

// The phase gradient into the internal real plane x_r (both gradient entry
// points; the caller has entered the plan's stream).
static int phase_gradient_internal(gswmtp_plan *p, const float *dev_g) {
  hipStream_t s = p->stream;
  HIP_TRY(p, ensure_forward(p, false));
  if (p->grid_form) {   // g Theta formed by the grid scatter itself
    HIP_TRY(p, scatter_products(p, p->b.theta, false, s, 1.f, dev_g));
  } else {
    HIP_TRY(p, launch_grad_field(p, dev_g, s));
    HIP_TRY(p, scatter_products(p, p->b.theta_new, false, s));
  }
  HIP_TRY(p, launch_cgemm(p, false, EPI_GRAD, p->b.s_r, p->b.s_i, p->b.x_r, p->b.x_i, p->b.p_r,
                          p->b.p_i, false, s));
  return GSWMTP_OK;
}

int gswmtp_phase_gradient_device(gswmtp_plan *p, const float *dev_g, float *dev_grad) {
  if (!p || !dev_g || !dev_grad) return GSWMTP_E_INVAL;
  if (is_split(p))
    return fail(p, GSWMTP_E_UNSUPPORTED, "phase gradient is built for FP32 plans only");
  DeviceGuard g(p->device);
  const Dims &D = p->d;
  HIP_TRY(p, enter(p));
  const int rc = phase_gradient_internal(p, dev_g);
  if (rc != GSWMTP_OK) return rc;
  hipLaunchKernelGGL(k_expand_real, grid1((size_t)D.ny * D.nx), dim3(256), 0, p->stream, p->b.x_r,
                     p->b.row_pos, p->b.col_pos, D.axis, D.ny, D.nx, D.Cp, dev_grad);
  HIP_TRY(p, hipGetLastError());
  HIP_TRY(p, leave(p));
  return GSWMTP_OK;
}

int gswmtp_phase_gradient_adam_device(gswmtp_plan *p, const float *dev_g, float *phi, float *m,
                                      float *v, const float *dev_step, double lr, double beta1,
                                      double beta2, double eps) {
  if (!p || !dev_g || !phi || !m || !v || !dev_step) return GSWMTP_E_INVAL;
  if (!std::isfinite(lr) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps >= 0.0) || !std::isfinite(eps))
    return GSWMTP_E_INVAL;
  if (is_split(p))
    return fail(p, GSWMTP_E_UNSUPPORTED, "phase gradient is built for FP32 plans only");
  DeviceGuard g(p->device);
  const Dims &D = p->d;
  HIP_TRY(p, enter(p));
  const int rc = phase_gradient_internal(p, dev_g);
  if (rc != GSWMTP_OK) return rc;
  const size_t np = (size_t)D.ny * D.nx;
  const auto aligned = [](const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  const bool vec = np % 4 == 0 && aligned(phi) && aligned(m) && aligned(v);
  const size_t groups = vec ? np / 4 : np;
  const dim3 grid((unsigned)std::min<size_t>((groups + 255) / 256, 8192));
  if (vec)
    hipLaunchKernelGGL(k_adam_internal<4>, grid, dim3(256), 0, p->stream, p->b.x_r,
                       p->b.row_pos, p->b.col_pos, D.axis, D.ny, D.nx, D.Cp, phi, m, v,
                       dev_step, (float)lr, (float)beta1, (float)beta2, (float)eps);
  else
    hipLaunchKernelGGL(k_adam_internal<1>, grid, dim3(256), 0, p->stream, p->b.x_r,
                       p->b.row_pos, p->b.col_pos, D.axis, D.ny, D.nx, D.Cp, phi, m, v,
                       dev_step, (float)lr, (float)beta1, (float)beta2, (float)eps);
  HIP_TRY(p, hipGetLastError());
  HIP_TRY(p, leave(p));
  return GSWMTP_OK;
}

int gswmtp_time_stages(gswmtp_plan *p, int n_iter, double *ms_out) {
  if (!p || n_iter < 1 || !ms_out) return GSWMTP_E_INVAL;
  DeviceGuard g(p->device);
  const int ne = (GSWMTP_N_STAGES + 1) * n_iter;
  std::vector<hipEvent_t> ev(ne, nullptr);
  for (auto &e : ev) HIP_TRY(p, hipEventCreate(&e));
  hipStream_t s = p->stream;
  int rc = GSWMTP_OK;
  do {
    if (enter(p) != hipSuccess) { rc = fail(p, GSWMTP_E_HIP, "enter"); break; }
    hipLaunchKernelGGL(k_control, dim3(1), dim3(1), 0, s, p->b.ctrl, p->b.stats, 0.0);
    for (int it = 0; it < n_iter && rc == GSWMTP_OK; ++it) {
      hipEvent_t *e = &ev[(size_t)it * (GSWMTP_N_STAGES + 1)];
      hipError_t er = hipEventRecord(e[0], s);
      if (er == hipSuccess) er = stage_forward(p, true, s);   // with the fused focus gather
      if (er == hipSuccess) er = hipEventRecord(e[1], s);
      if (er == hipSuccess) er = launch_update(p, UPD_ITERATE, s);
      if (er == hipSuccess) er = hipEventRecord(e[2], s);
      if (er == hipSuccess) er = stage_scatter(p, true, s);
      if (er == hipSuccess) er = hipEventRecord(e[3], s);
      if (er == hipSuccess) er = stage_adjoint(p, true, s, 1);
      if (er == hipSuccess) er = hipEventRecord(e[4], s);
      if (er == hipSuccess) er = stage_adjoint(p, true, s, 2);
      if (er == hipSuccess) er = hipEventRecord(e[5], s);
      if (er != hipSuccess) rc = fail(p, GSWMTP_E_HIP, "time_stages launch", er);
    }
    if (rc != GSWMTP_OK) break;
    if (hipStreamSynchronize(s) != hipSuccess) { rc = fail(p, GSWMTP_E_HIP, "sync"); break; }
    for (int k = 0; k < GSWMTP_N_STAGES; ++k) ms_out[k] = 0.0;
    for (int it = 0; it < n_iter; ++it) {
      hipEvent_t *e = &ev[(size_t)it * (GSWMTP_N_STAGES + 1)];
      for (int k = 0; k < GSWMTP_N_STAGES; ++k) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e[k], e[k + 1]);
        ms_out[k] += ms / n_iter;
      }
    }
    p->fwd_valid = p->stats_valid = false;
    if (leave(p) != hipSuccess) rc = fail(p, GSWMTP_E_HIP, "leave");
  } while (false);
  for (auto &e : ev)
    if (e) (void)hipEventDestroy(e);
  return rc;
}

const char *gswmtp_stage_kernel(gswmtp_plan *p, int stage) {
  if (!p) return "";
  const bool split = is_split(p);
  switch (stage) {
    case 0: return cgemm_kernel_name(p, true, EPI_GATHER);
    case 1: return "focus_update";
    case 2:
      if (p->scaled_adj) return "k_scale_adjoint_split";
      return split ? "focus_scatter_split" : "focus_scatter";
    case 3: return cgemm_kernel_name(p, false, EPI_PROJECT);
    case 4:
      if (p->sched_bwd.n_tail == 0) return "";
      return split ? "cgemm_tail_project_split" : "cgemm_tail_project";
  }
  return "";
}

}  // extern "C"

int gswmtp::fault_alloc_setting() {
  const char *v = std::getenv("GSWMTP_FAULT_INJECT");
  if (!v || std::strncmp(v, "alloc", 5) != 0) return -1;
  if (v[5] == '\0') return 0;
  if (v[5] != ':') return -1;
  char *end = nullptr;
  const long k = std::strtol(v + 6, &end, 10);
  return (end && *end == '\0' && k >= 1 && k <= 1000) ? (int)k : -1;
}

bool gswmtp::fault_alloc_hit(int setting, int *count) {
  const int n = ++*count;
  return setting == 0 || (setting > 0 && n == setting);
}
