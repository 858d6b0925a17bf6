/*
 * FP64 CPU oracle for the weighted Gerchberg-Saxton iteration whose
 * diffraction operator is the matrix triple product (MTP) of
 * Liu et al., "Fast generation of arbitrary optical focus array",
 * arXiv:2206.12661.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark build, load or call this file.  The GPU
 * library never links, includes or calls it, and this file includes nothing
 * of the GPU library.
 *
 * What it computes, all in double precision:
 *
 *  - Forward propagation (Eq. 1 sampled on the pupil, written in the separable
 *    form of Eq. 2): for every focus n,
 *        Theta_n = sum_j sum_i E[j][i] exp(-2 pi i s_y v_j y_n) exp(-2 pi i s_x u_i x_n).
 *    The sum runs over every pupil sample and every focus separately: there is
 *    no deduplication of focal coordinates and no aperture compaction, so this
 *    checks the GPU's reduced-grid evaluation independently.
 *
 *  - Inverse propagation: the paper only says the inverse operator is
 *    formulated like the forward one.  It is read here as the adjoint
 *    (conjugate transpose) of the forward map with zero focal field at every
 *    point that is not a focus:
 *        E'[j][i] = sum_n Theta'_n exp(+2 pi i s_y v_j y_n) exp(+2 pi i s_x u_i x_n).
 *
 *  - The iteration of Algorithm 1 ("Fast generation of arbitrary OFA"), step
 *    by step: forward propagation, focus intensities, intensity accuracy,
 *    termination test, weight update, focal-field update, inverse
 *    propagation, phase-only projection.  Where the paper leaves a choice open
 *    the reading taken is stated at the step.
 *
 * Parallelism: OpenMP over foci (forward) and pupil rows (adjoint).  Every
 * output element is summed by one thread in a fixed order, so results do not
 * depend on the thread count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Smallest normalised intensity used in the weight update (division guard). */
#define ORACLE_TAU 1e-30

/* exp(-2 pi i s c f) exp(i pi z (s c)^2) for every sample coordinate c, one
 * focal coordinate f at axial position z.  The first factor follows Eq. 1
 * (negative sign in the forward direction); the second is the defocus phase
 * of the pupil that places a focus off the focal plane (Sec. 3: the axial
 * position of a focus is set by a defocus phase of the pupil function),
 * separable over the two pupil axes; z = 0 is the focal plane. */
static void phasor_row(int n, const double *coord, double s, double f, double z,
                       double *re, double *im)
{
    for (int p = 0; p < n; ++p) {
        double sc = s * coord[p];
        double arg = -2.0 * M_PI * sc * f + M_PI * z * sc * sc;
        re[p] = cos(arg);
        im[p] = sin(arg);
    }
}

/* Per-focus phasor tables: ax[n][i] and ay[n][j]. */
typedef struct {
    int nf, nx, ny;
    double *axr, *axi, *ayr, *ayi;
} tables;

static int tables_build(tables *t, int ny, int nx, const double *u, const double *v,
                        double sx, double sy, int nf, const double *fx, const double *fy,
                        const double *fz)
{
    t->nf = nf; t->nx = nx; t->ny = ny;
    t->axr = malloc(sizeof(double) * (size_t)nf * nx);
    t->axi = malloc(sizeof(double) * (size_t)nf * nx);
    t->ayr = malloc(sizeof(double) * (size_t)nf * ny);
    t->ayi = malloc(sizeof(double) * (size_t)nf * ny);
    if (!t->axr || !t->axi || !t->ayr || !t->ayi) return -1;
#pragma omp parallel for schedule(static)
    for (int n = 0; n < nf; ++n) {
        const double z = fz ? fz[n] : 0.0;
        phasor_row(nx, u, sx, fx[n], z, t->axr + (size_t)n * nx, t->axi + (size_t)n * nx);
        phasor_row(ny, v, sy, fy[n], z, t->ayr + (size_t)n * ny, t->ayi + (size_t)n * ny);
    }
    return 0;
}

static void tables_free(tables *t)
{
    free(t->axr); free(t->axi); free(t->ayr); free(t->ayi);
}

/* Forward propagation with prebuilt tables.  E is interleaved complex
 * [ny][nx]; theta is interleaved complex [nf]. */
static void forward_t(const tables *t, const double *E, double *theta)
{
    const int nx = t->nx, ny = t->ny;
#pragma omp parallel for schedule(dynamic, 1)
    for (int n = 0; n < t->nf; ++n) {
        const double *axr = t->axr + (size_t)n * nx, *axi = t->axi + (size_t)n * nx;
        const double *ayr = t->ayr + (size_t)n * ny, *ayi = t->ayi + (size_t)n * ny;
        double tr = 0.0, ti = 0.0;
        for (int j = 0; j < ny; ++j) {
            const double *row = E + 2 * (size_t)j * nx;
            double rr = 0.0, ri = 0.0;          /* sum_i E[j][i] ax[i] */
            for (int i = 0; i < nx; ++i) {
                double er = row[2 * i], ei = row[2 * i + 1];
                rr += er * axr[i] - ei * axi[i];
                ri += er * axi[i] + ei * axr[i];
            }
            tr += ayr[j] * rr - ayi[j] * ri;    /* ... times ay[j] */
            ti += ayr[j] * ri + ayi[j] * rr;
        }
        theta[2 * n] = tr;
        theta[2 * n + 1] = ti;
    }
}

/* Adjoint with prebuilt tables: E'[j][i] = sum_n theta_n conj(ay[n][j]) conj(ax[n][i]). */
static void adjoint_t(const tables *t, const double *theta, double *E)
{
    const int nx = t->nx, ny = t->ny;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < ny; ++j) {
        double *row = E + 2 * (size_t)j * nx;
        memset(row, 0, sizeof(double) * 2 * (size_t)nx);
        for (int n = 0; n < t->nf; ++n) {
            double ayr = t->ayr[(size_t)n * ny + j], ayi = -t->ayi[(size_t)n * ny + j];
            double cr = theta[2 * n] * ayr - theta[2 * n + 1] * ayi;
            double ci = theta[2 * n] * ayi + theta[2 * n + 1] * ayr;
            const double *axr = t->axr + (size_t)n * nx, *axi = t->axi + (size_t)n * nx;
            for (int i = 0; i < nx; ++i) {      /* times conj(ax[n][i]) */
                row[2 * i] += cr * axr[i] + ci * axi[i];
                row[2 * i + 1] += ci * axr[i] - cr * axi[i];
            }
        }
    }
}

/* Threads of the OpenMP loops (n >= 1); results do not depend on it. */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Forward propagation, Eq. 1 / Eq. 2, evaluated at the foci. */
int oracle_forward(int ny, int nx, const double *E, const double *u, const double *v,
                   double sx, double sy, int nf, const double *fx, const double *fy,
                   const double *fz, double *theta)
{
    tables t;
    if (tables_build(&t, ny, nx, u, v, sx, sy, nf, fx, fy, fz)) { tables_free(&t); return -1; }
    forward_t(&t, E, theta);
    tables_free(&t);
    return 0;
}

/* Inverse propagation read as the adjoint of the forward map. */
int oracle_adjoint(int ny, int nx, const double *u, const double *v, double sx, double sy,
                   int nf, const double *fx, const double *fy, const double *fz,
                   const double *theta, double *E)
{
    tables t;
    if (tables_build(&t, ny, nx, u, v, sx, sy, nf, fx, fy, fz)) { tables_free(&t); return -1; }
    adjoint_t(&t, theta, E);
    tables_free(&t);
    return 0;
}

/* Focus statistics of one forward field (Algorithm 1, intensity and accuracy;
 * efficiency and uniformity as diagnostics).
 *   I_n = |Theta_n|^2, i = I / sum I, t = target / sum target.
 *   accuracy   xi  = 1 - ||t - i||_2 / ||i||_2.  The paper writes the norm of
 *              (target - I) over the norm of I; both intensities are taken
 *              normalised to unit sum so that the measure does not depend on
 *              the arbitrary scale of the computed field.
 *   efficiency eta = sum I / (N_ap * sum A^2): the fraction of the incident
 *              power that reaches the foci, relative to the peak a single focus
 *              can reach under the same pupil (equality by Cauchy-Schwarz).
 *   uniformity  U  = 1 - (max r - min r) / (max r + min r), r_n = i_n / t_n over
 *              foci with a positive target.
 * out[0..2] = xi, eta, U; out[3] = sum I. */
void oracle_stats(int nf, const double *theta, const double *target, double n_ap,
                  double sum_a2, double *out)
{
    double sI = 0.0, sT = 0.0;
    for (int n = 0; n < nf; ++n) {
        sI += theta[2 * n] * theta[2 * n] + theta[2 * n + 1] * theta[2 * n + 1];
        sT += target[n];
    }
    double d2 = 0.0, i2 = 0.0, rmax = -INFINITY, rmin = INFINITY;
    for (int n = 0; n < nf; ++n) {
        double I = theta[2 * n] * theta[2 * n] + theta[2 * n + 1] * theta[2 * n + 1];
        double in = sI > 0.0 ? I / sI : 0.0;
        double tn = target[n] / sT;
        d2 += (tn - in) * (tn - in);
        i2 += in * in;
        if (tn > 0.0) {
            double r = in / tn;
            if (r > rmax) rmax = r;
            if (r < rmin) rmin = r;
        }
    }
    out[0] = i2 > 0.0 ? 1.0 - sqrt(d2) / sqrt(i2) : -INFINITY;
    out[1] = sI / (n_ap * sum_a2);
    out[2] = (rmax + rmin) > 0.0 ? 1.0 - (rmax - rmin) / (rmax + rmin) : 0.0;
    out[3] = sI;
}

/* Phase-only projection of Algorithm 1: phi = arg E' where A > 0 (0 elsewhere
 * and where E' = 0), range (-pi, pi]; then E = A exp(i phi). */
void oracle_project(int np, const double *amp, const double *Ep, double *phi, double *E)
{
    for (int p = 0; p < np; ++p) {
        double ph = 0.0;
        if (amp[p] > 0.0 && (Ep[2 * p] != 0.0 || Ep[2 * p + 1] != 0.0)) {
            ph = atan2(Ep[2 * p + 1], Ep[2 * p]);
            if (ph == -M_PI) ph = M_PI;
        }
        phi[p] = ph;
        E[2 * p] = amp[p] * cos(ph);
        E[2 * p + 1] = amp[p] * sin(ph);
    }
}

/* Weight update and focal-field update of one pass (Algorithm 1), with the
 * variants of Sec. 2:
 *   weighting 0 (GSW, Algorithm 1): w <- w sqrt(t / max(i, tau)), where
 *   t = target / sum target and i = I / sum I.  The ratio uses these
 *   unit-sum intensities (the paper's raw target / I ratio would shrink every
 *   weight by the arbitrary field scale at every pass); tau keeps it finite
 *   when a focus is dark;
 *   weighting 1 (plain GS, the comparison method): w unchanged;
 *   phasor: arg Theta of this pass, or, when fixed != NULL, the stored
 *   phasors (phase fixing: the focal phases are frozen);
 *   measured (nullable): intensities captured by a camera for this pass's
 *   phase (the camera-in-the-loop strategy of the experiments in Sec. 2):
 *   the weight update takes i from them (normalised to unit sum) instead of
 *   from |Theta|^2; the phasors still come from Theta.
 * theta_new = w sqrt(target) * phasor (phasor 1 where Theta_n = 0).  This is
 * the one implementation of the update: the iteration, the measured pass and
 * oracle_weight_update all call it. */
void oracle_weight_update_ex(int nf, const double *theta, const double *target, double *w,
                             double *theta_new, int weighting, const double *fixed,
                             const double *measured)
{
    double sI = 0.0, sT = 0.0;
    for (int n = 0; n < nf; ++n) {
        sI += measured ? measured[n]
                       : theta[2 * n] * theta[2 * n] + theta[2 * n + 1] * theta[2 * n + 1];
        sT += target[n];
    }
    for (int n = 0; n < nf; ++n) {
        double re = theta[2 * n], im = theta[2 * n + 1];
        double I = re * re + im * im;
        if (weighting == 0) {
            double Iw = measured ? measured[n] : I;
            double in = sI > 0.0 ? Iw / sI : 0.0;
            double tn = target[n] / sT;
            w[n] *= sqrt(tn / (in > ORACLE_TAU ? in : ORACLE_TAU));
        }
        double pr = 1.0, pi = 0.0;
        if (fixed) {
            pr = fixed[2 * n];
            pi = fixed[2 * n + 1];
        } else {
            double mag = sqrt(I);
            if (mag > 0.0) { pr = re / mag; pi = im / mag; }
        }
        double a = w[n] * sqrt(target[n]);
        theta_new[2 * n] = a * pr;
        theta_new[2 * n + 1] = a * pi;
    }
}

/* Weight update and focal-field update of Algorithm 1 as printed (GSW
 * weighting, phasors of this pass, computed intensities): the same function
 * every pass of the iteration below runs. */
void oracle_weight_update(int nf, const double *theta, const double *target, double *w,
                          double *theta_new)
{
    oracle_weight_update_ex(nf, theta, target, w, theta_new, 0, NULL, NULL);
}

/* Phasors arg Theta_n (1 where Theta_n = 0). */
static void phasors(int nf, const double *theta, double *out)
{
    for (int n = 0; n < nf; ++n) {
        double re = theta[2 * n], im = theta[2 * n + 1];
        double mag = sqrt(re * re + im * im);
        out[2 * n] = mag > 0.0 ? re / mag : 1.0;
        out[2 * n + 1] = mag > 0.0 ? im / mag : 0.0;
    }
}

/* Algorithm 1 with the variants of Sec. 2.  phi: in = initial phase, out =
 * phase after the run.  w: in/out weights (pass ones for a fresh start).
 * hist (nullable): 3 doubles per pass (xi, eta, U of that pass's forward
 * field).  The termination test (xi > stop, disabled when stop <= 0) runs
 * before the update, so a stopping pass leaves phi unchanged and is not
 * counted in iters_done.  theta_final (nullable) receives the field of the
 * returned phase.  weighting: 0 GSW, 1 GS.  phase_fix > 0: the focal phases
 * are frozen from the phase_fix-th updating pass on (the phasors of that
 * pass's forward field are recorded and used by it and every later pass;
 * <= 0 disables).  Returns 0, or -1 on allocation failure. */
int oracle_gsw_ex(int ny, int nx, const double *amp, const double *u, const double *v,
                  double sx, double sy, int nf, const double *fx, const double *fy,
                  const double *fz, const double *target, double *phi, double *w, int n_iter, double stop,
                  double *hist, int *iters_done, double *theta_final, int weighting,
                  int phase_fix)
{
    const size_t np = (size_t)ny * nx;
    tables t;
    double *E = malloc(sizeof(double) * 2 * np);
    double *Ep = malloc(sizeof(double) * 2 * np);
    double *th = malloc(sizeof(double) * 2 * (size_t)nf);
    double *thn = malloc(sizeof(double) * 2 * (size_t)nf);
    double *fix = malloc(sizeof(double) * 2 * (size_t)nf);
    int rc = -1;
    if (!E || !Ep || !th || !thn || !fix) goto done;
    if (tables_build(&t, ny, nx, u, v, sx, sy, nf, fx, fy, fz)) { tables_free(&t); goto done; }

    double n_ap = 0.0, sum_a2 = 0.0;
    for (size_t p = 0; p < np; ++p) {
        if (amp[p] > 0.0) n_ap += 1.0;
        sum_a2 += amp[p] * amp[p];
    }
    /* Initial pupil function E0 = A exp(i phi0). */
    for (size_t p = 0; p < np; ++p) {
        E[2 * p] = amp[p] * cos(phi[p]);
        E[2 * p + 1] = amp[p] * sin(phi[p]);
    }
    int done_passes = 0, recorded = 0;
    for (int it = 0; it < n_iter; ++it) {
        forward_t(&t, E, th);                         /* forward propagation */
        double st[4];
        oracle_stats(nf, th, target, n_ap, sum_a2, st); /* intensity, accuracy */
        if (hist) { hist[3 * it] = st[0]; hist[3 * it + 1] = st[1]; hist[3 * it + 2] = st[2]; }
        if (stop > 0.0 && st[0] > stop) break;        /* termination test */
        const int j = done_passes + 1;                /* this updating pass, from 1 */
        if (phase_fix > 0 && j >= phase_fix && !recorded) {
            phasors(nf, th, fix);                     /* freeze the focal phases */
            recorded = 1;
        }
        oracle_weight_update_ex(nf, th, target, w, thn, weighting, recorded ? fix : NULL, NULL);
        adjoint_t(&t, thn, Ep);                       /* inverse propagation */
        oracle_project((int)np, amp, Ep, phi, E);            /* phase-only constraint */
        ++done_passes;
    }
    if (iters_done) *iters_done = done_passes;
    if (theta_final) forward_t(&t, E, theta_final);
    tables_free(&t);
    rc = 0;
done:
    free(E); free(Ep); free(th); free(thn); free(fix);
    return rc;
}

/* One pass of Algorithm 1 (GSW weighting) whose weight update uses measured
 * focus intensities (camera in the loop, Sec. 2 experiments): forward field
 * of phi, its statistics into hist3 (nullable, xi / eta / U of the computed
 * field), weight update with i = measured / sum(measured), new focal field
 * w sqrt(target) arg Theta, adjoint, phase-only projection.  phi and w are
 * updated in place.  Returns 0, or -1 on allocation failure. */
int oracle_gsw_measured_pass(int ny, int nx, const double *amp, const double *u, const double *v,
                             double sx, double sy, int nf, const double *fx, const double *fy,
                             const double *fz, const double *target, double *phi, double *w,
                             const double *measured, double *hist3)
{
    const size_t np = (size_t)ny * nx;
    tables t;
    double *E = malloc(sizeof(double) * 2 * np);
    double *Ep = malloc(sizeof(double) * 2 * np);
    double *th = malloc(sizeof(double) * 2 * (size_t)nf);
    double *thn = malloc(sizeof(double) * 2 * (size_t)nf);
    int rc = -1;
    if (!E || !Ep || !th || !thn) goto done;
    if (tables_build(&t, ny, nx, u, v, sx, sy, nf, fx, fy, fz)) { tables_free(&t); goto done; }
    double n_ap = 0.0, sum_a2 = 0.0;
    for (size_t p = 0; p < np; ++p) {
        if (amp[p] > 0.0) n_ap += 1.0;
        sum_a2 += amp[p] * amp[p];
        E[2 * p] = amp[p] * cos(phi[p]);
        E[2 * p + 1] = amp[p] * sin(phi[p]);
    }
    forward_t(&t, E, th);
    double st[4];
    oracle_stats(nf, th, target, n_ap, sum_a2, st);
    if (hist3) { hist3[0] = st[0]; hist3[1] = st[1]; hist3[2] = st[2]; }
    oracle_weight_update_ex(nf, th, target, w, thn, 0, NULL, measured);
    adjoint_t(&t, thn, Ep);
    oracle_project((int)np, amp, Ep, phi, E);
    tables_free(&t);
    rc = 0;
done:
    free(E); free(Ep); free(th); free(thn);
    return rc;
}

/* Algorithm 1 as printed (GSW weighting, no phase fixing). */
int oracle_gsw(int ny, int nx, const double *amp, const double *u, const double *v,
               double sx, double sy, int nf, const double *fx, const double *fy,
               const double *target, double *phi, double *w, int n_iter, double stop,
               double *hist, int *iters_done, double *theta_final)
{
    return oracle_gsw_ex(ny, nx, amp, u, v, sx, sy, nf, fx, fy, NULL, target, phi, w, n_iter,
                         stop, hist, iters_done, theta_final, 0, 0);
}

/* Gradient of L(phi) = sum_n g_n I_n(phi) with I_n = |Theta_n|^2 and
 * E = A exp(i phi):
 *   dL/dphi_p = 2 Im( conj(E_p) * [adjoint(g * Theta)]_p ).
 * theta (nullable) receives the forward field at phi. */
int oracle_phase_gradient(int ny, int nx, const double *amp, const double *u, const double *v,
                          double sx, double sy, int nf, const double *fx, const double *fy, const double *fz,
                          const double *phi, const double *g, double *grad, double *theta)
{
    const size_t np = (size_t)ny * nx;
    tables t;
    double *E = malloc(sizeof(double) * 2 * np);
    double *Ep = malloc(sizeof(double) * 2 * np);
    double *th = malloc(sizeof(double) * 2 * (size_t)nf);
    int rc = -1;
    if (!E || !Ep || !th) goto done;
    if (tables_build(&t, ny, nx, u, v, sx, sy, nf, fx, fy, fz)) { tables_free(&t); goto done; }
    for (size_t p = 0; p < np; ++p) {
        E[2 * p] = amp[p] * cos(phi[p]);
        E[2 * p + 1] = amp[p] * sin(phi[p]);
    }
    forward_t(&t, E, th);
    if (theta) memcpy(theta, th, sizeof(double) * 2 * (size_t)nf);
    for (int n = 0; n < nf; ++n) { th[2 * n] *= g[n]; th[2 * n + 1] *= g[n]; }
    adjoint_t(&t, th, Ep);
    for (size_t p = 0; p < np; ++p)
        grad[p] = 2.0 * (E[2 * p] * Ep[2 * p + 1] - E[2 * p + 1] * Ep[2 * p]);
    tables_free(&t);
    rc = 0;
done:
    free(E); free(Ep); free(th);
    return rc;
}
