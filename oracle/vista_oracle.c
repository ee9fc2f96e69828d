/*
 * FP64 CPU oracle for the ViSta stacking hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference the GPU library is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it; the product library
 * never does.  It shares no code, header or table with the GPU path.
 *
 * What it computes (Torsello et al., "The ViSta method ...", Proc. SPIE 14153):
 *   for every target, row, channel and polarisation, in that order,
 *     - the channel is moved to the rest frame, nu_rest = nu_obs (1+z) (Sec. 3.1);
 *     - the uvw are taken to wavelengths at the sample's own frequency,
 *       u_lambda = u_m nu_obs / c, which is the 1/(1+z) baseline scaling of Eq. 1
 *       paired with the rest-frame frequency;
 *     - the visibility is multiplied by the phase-centre shift of Eq. 2, with
 *       (dl, dm, dn) = (0 - l, 0 - m, 1 - n), i.e. by exp(+2 pi i t),
 *       t = u l + v m + w (n - 1) in turns;
 *     - the rotated value is split over the common rest channels with the
 *       channel-overlap weights of Eq. 3-4 (input width: the given width, else a
 *       centred finite difference, one-sided at the ends);
 *     - each (weight * fraction)-weighted value is added to the nearest uv cell of a
 *       common (u, v, nu_rest) grid holding sum(w f V'), sum(w f), the number of
 *       contributions and sum(w f |V'|) (the last is only a scale for error norms).
 *   The paper casts visibilities to double before the phase multiply (Sec. 3.2, last
 *   paragraph); so does this file, and everything else is double too.
 *
 * With a target's rotation switched on (Eq. 1's R from the phase centre to the stacking
 * position, given as two (R.A., Dec.) pairs), (l, m) are the stacking position's
 * direction cosines and the uv cell is taken from the rotated baseline R (u, v, w); the
 * Eq. 2 phase still uses the original baseline (its turns are exactly w' - w).
 *
 * It also computes the paper's own per-row product (ora_rebin_window, ora_rebin_rows):
 * each target's rows rebinned onto the target's own output window by Eq. 3 with the
 * Eq. 4 weights, normalised per row and output channel, after the same Eq. 2 shift, and
 * its baseline R (u, v, w) / (1 + z) (Eq. 1).
 *
 * Build with -ffp-contract=off and without fast-math: the cell and channel indices
 * must follow exactly the operation sequence written here.
 *
 * Parallelism: ora_stack splits the requested rest-channel range into contiguous
 * slabs, one per OpenMP thread.  Each cell is owned by one thread, which adds its
 * contributions in (target, row, channel, polarisation) order, so the result does
 * not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_C 299792458.0
#define ORA_SLIVER 1e-9
#define ORA_PI 3.14159265358979323846
#define ORA_NEAREST 4u          /* grid flag: one output channel per input channel */

typedef struct {
    int32_t nu, nv, nchan;
    double du, dv, freq_lo, dfreq;
    uint32_t flags;
} ora_grid;

typedef struct {
    int64_t nrow;
    int32_t nchan, npol;
    const double* uvw;        /* [nrow][3] metres */
    const float* vis;         /* [nrow][nk][npol][2] (re, im) */
    const float* weight;      /* [nrow][npol], or [nrow][nk][npol] if weight_per_chan */
    const uint8_t* flag;      /* [nrow][nk][npol] or NULL */
    const double* chan_freq;  /* [nchan], all channels */
    const double* chan_width; /* [nchan] or NULL */
    double l, m, z;
    int32_t weight_per_chan;
    int32_t kbeg, kend;       /* the channels [kbeg, kend) are the ones used */
    int32_t rotate;           /* 1: Eq. 1's rotation from (ra0, dec0) to (ra1, dec1) [rad];
                                 l, m are then taken from the angles */
    double ra0, dec0, ra1, dec1;
    int32_t kdata, kstride;   /* the data arrays hold channels [kdata, kdata + kstride) of
                                 each row, nk = kstride; kstride == 0: they hold exactly
                                 [kbeg, kend) (kdata = kbeg, nk = kend - kbeg) */
} ora_target;

/* Position of sample (r, k, p) in the data arrays (indexing only). */
static size_t ora_elem(const ora_target* t, int64_t r, int32_t k, int32_t p) {
    const int32_t k0 = t->kstride > 0 ? t->kdata : t->kbeg;
    const int32_t nk = t->kstride > 0 ? t->kstride : t->kend - t->kbeg;
    return ((size_t)r * (size_t)nk + (size_t)(k - k0)) * (size_t)t->npol + (size_t)p;
}

/* Per-channel rest-frame table of one target: a_k = nu_k / c and the contributing set
 * J_k = {(j, f_kj)} stored as a CSR list. */
typedef struct {
    int32_t nchan;
    double* a;        /* [nchan] */
    double* width;    /* [nchan] W_k */
    double* lo;       /* [nchan] rest-frame lower edge */
    double* hi;       /* [nchan] rest-frame upper edge */
    int32_t* start;   /* [nchan+1] */
    int32_t* j;       /* [start[nchan]] */
    double* f;        /* [start[nchan]] */
} ora_table;

/* Input channel width W_k (Eq. 4's Delta nu_k): the given width, else a centred
 * finite difference |nu_{k+1} - nu_{k-1}| / 2, one-sided at the two ends. */
static double ora_width(const double* f, const double* w, int32_t n, int32_t k) {
    if (w) return w[k];
    if (n < 2) return NAN;
    if (k == 0) return fabs(f[1] - f[0]);
    if (k == n - 1) return fabs(f[n - 1] - f[n - 2]);
    return fabs(f[k + 1] - f[k - 1]) / 2.0;
}

/* Build the table of one target (Sec. 3.1 rest frame; Eq. 3-4 overlaps). */
static int ora_build_table(const ora_grid* g, const ora_target* t, ora_table* tb) {
    int32_t n = t->nchan;
    double opz = 1.0 + t->z;
    int32_t cap = 0, k, j;
    memset(tb, 0, sizeof(*tb));
    tb->nchan = n;
    tb->a = (double*)malloc(sizeof(double) * n);
    tb->width = (double*)malloc(sizeof(double) * n);
    tb->lo = (double*)malloc(sizeof(double) * n);
    tb->hi = (double*)malloc(sizeof(double) * n);
    tb->start = (int32_t*)malloc(sizeof(int32_t) * (n + 1));
    if (!tb->a || !tb->width || !tb->lo || !tb->hi || !tb->start) return -3;
    for (k = 0; k < n; ++k) {
        double W = ora_width(t->chan_freq, t->chan_width, n, k);
        tb->a[k] = t->chan_freq[k] / ORA_C;
        tb->width[k] = W;
        tb->lo[k] = (t->chan_freq[k] - 0.5 * W) * opz;
        tb->hi[k] = (t->chan_freq[k] + 0.5 * W) * opz;
    }
    /* Two passes over every (k, j): count, then fill. */
    for (int pass = 0; pass < 2; ++pass) {
        int32_t pos = 0;
        for (k = 0; k < n; ++k) {
            tb->start[k] = pos;
            if (g->flags & ORA_NEAREST) {
                double x = floor((t->chan_freq[k] * opz - g->freq_lo) / g->dfreq);
                if (x >= 0.0 && x < (double)g->nchan) {
                    if (pass) { tb->j[pos] = (int32_t)x; tb->f[pos] = 1.0; }
                    ++pos;
                }
                continue;
            }
            double Wr = tb->width[k] * opz;
            for (j = 0; j < g->nchan; ++j) {
                double e0 = g->freq_lo + (double)j * g->dfreq;
                double e1 = g->freq_lo + (double)(j + 1) * g->dfreq;
                double ov = fmin(tb->hi[k], e1) - fmax(tb->lo[k], e0);
                double f = ov / Wr;
                if (f > ORA_SLIVER) {
                    if (pass) { tb->j[pos] = j; tb->f[pos] = f; }
                    ++pos;
                }
            }
        }
        tb->start[n] = pos;
        if (!pass) {
            cap = pos > 0 ? pos : 1;
            tb->j = (int32_t*)malloc(sizeof(int32_t) * cap);
            tb->f = (double*)malloc(sizeof(double) * cap);
            if (!tb->j || !tb->f) return -3;
        }
    }
    return 0;
}

static void ora_free_table(ora_table* tb) {
    free(tb->a); free(tb->width); free(tb->lo); free(tb->hi);
    free(tb->start); free(tb->j); free(tb->f);
    memset(tb, 0, sizeof(*tb));
}

/* n - 1 for direction cosines (l, m), in the form free of cancellation:
 * sqrt(1-q) - 1 = -q / (1 + sqrt(1-q)), q = l^2 + m^2. */
static double ora_n_minus_1(double l, double m) {
    double q = l * l + m * m;
    return -q / (1.0 + sqrt(1.0 - q));
}

/* Eq. 1's rotation R.  The uvw frame of a phase centre (ra, dec) has, in equatorial
 * coordinates, the axes u = (-sin ra, cos ra, 0) (east), v = (-sin dec cos ra,
 * -sin dec sin ra, cos dec) (north) and w = (cos dec cos ra, cos dec sin ra, sin dec)
 * (towards the centre).  A baseline with coordinates (u, v, w) about the phase centre
 * (ra0, dec0) has coordinates R (u, v, w) about the stacking position (ra1, dec1), with
 * R[i][j] = axis_i(ra1, dec1) . axis_j(ra0, dec0); R's third row is the stacking
 * position's direction cosines (l, m, n) about the phase centre, so w' - w is exactly
 * the Eq. 2 turns u l + v m + w (n - 1).  Without the rotation R is the identity and
 * (l, m) are the target's given direction cosines. */
typedef struct {
    int rotate;
    double R[9];
    double l, m, nm1;
} ora_frame;

static void ora_axes(double ra, double dec, double ax[3][3]) {
    ax[0][0] = -sin(ra);            ax[0][1] = cos(ra);             ax[0][2] = 0.0;
    ax[1][0] = -sin(dec) * cos(ra); ax[1][1] = -sin(dec) * sin(ra); ax[1][2] = cos(dec);
    ax[2][0] = cos(dec) * cos(ra);  ax[2][1] = cos(dec) * sin(ra);  ax[2][2] = sin(dec);
}

static void ora_make_frame(const ora_target* t, ora_frame* f) {
    f->rotate = t->rotate;
    if (t->rotate) {
        double a0[3][3], a1[3][3];
        ora_axes(t->ra0, t->dec0, a0);
        ora_axes(t->ra1, t->dec1, a1);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                f->R[3 * i + j] = a1[i][0] * a0[j][0] + a1[i][1] * a0[j][1] + a1[i][2] * a0[j][2];
        f->l = f->R[6];
        f->m = f->R[7];
    } else {
        for (int i = 0; i < 9; ++i) f->R[i] = (i % 4 == 0) ? 1.0 : 0.0;
        f->l = t->l;
        f->m = t->m;
    }
    f->nm1 = ora_n_minus_1(f->l, f->m);
}

/* The baseline about the stacking position: R (u, v, w). */
static void ora_rot(const ora_frame* f, const double* uvw, double* out) {
    if (!f->rotate) {
        out[0] = uvw[0]; out[1] = uvw[1]; out[2] = uvw[2];
        return;
    }
    for (int i = 0; i < 3; ++i) out[i] = f->R[3 * i] * uvw[0] + f->R[3 * i + 1] * uvw[1] + f->R[3 * i + 2] * uvw[2];
}

/* Nearest uv cell of a (row, channel): u = u_m a_k in wavelengths, index
 * rint(u / du) counted from the centre cell n/2.  The bounds test is made on the
 * rounded value in double, so a non-finite or huge coordinate is simply outside;
 * iu/iv get INT64_MIN when the rounded value does not fit.  Returns 1 if inside. */
static int ora_cell(const ora_grid* g, const double* uvw_row, double a, int64_t* iu, int64_t* iv) {
    double inv_du = 1.0 / g->du, inv_dv = 1.0 / g->dv;
    double u = uvw_row[0] * a;
    double v = uvw_row[1] * a;
    double ru = rint(u * inv_du);
    double rv = rint(v * inv_dv);
    *iu = fabs(ru) < 4.0e18 ? (int64_t)ru + g->nu / 2 : INT64_MIN;
    *iv = fabs(rv) < 4.0e18 ? (int64_t)rv + g->nv / 2 : INT64_MIN;
    return ru >= -(double)(g->nu / 2) && ru < (double)(g->nu - g->nu / 2) &&
           rv >= -(double)(g->nv / 2) && rv < (double)(g->nv - g->nv / 2);
}

/* Eq. 2 phasor: exp(+2 pi i t) with t = u l + v m + w (n-1) in turns, reduced to
 * t - rint(t) before the trigonometry. */
static void ora_phasor(const double* uvw_row, double a, double l, double m, double nm1,
                       double* c, double* s) {
    double u = uvw_row[0] * a, v = uvw_row[1] * a, w = uvw_row[2] * a;
    double t = u * l + v * m + w * nm1;
    double ph = 2.0 * ORA_PI * (t - rint(t));
    *c = cos(ph);
    *s = sin(ph);
}

static double ora_weight(const ora_target* t, int64_t r, int32_t k, int32_t p) {
    if (t->weight_per_chan) return (double)t->weight[ora_elem(t, r, k, p)];
    return (double)t->weight[(size_t)r * t->npol + p];
}

/* ------------------------------------------------------------------------------- */

int ora_check(const ora_grid* g, int32_t ntgt, const ora_target* tg) {
    if (!g || g->nu < 1 || g->nv < 1 || g->nchan < 1) return -1;
    if (!(g->du > 0 && isfinite(g->du) && g->dv > 0 && isfinite(g->dv))) return -1;
    if (!(g->dfreq > 0 && isfinite(g->dfreq) && isfinite(g->freq_lo))) return -1;
    for (int32_t i = 0; i < ntgt; ++i) {
        const ora_target* t = &tg[i];
        if (t->nrow < 0 || t->nchan < 1 || (t->npol != 1 && t->npol != 2 && t->npol != 4)) return -1;
        if (t->kbeg < 0 || t->kend > t->nchan || t->kbeg > t->kend) return -1;
        if (t->kstride < 0) return -1;
        if (t->kstride > 0 && (t->kdata < 0 || t->kdata > t->kbeg || t->kend > t->kdata + t->kstride ||
                               t->kdata + t->kstride > t->nchan)) return -1;
        if (t->nchan == 1 && !t->chan_width) return -1;
        if (!(t->z > -1.0 && isfinite(t->z))) return -1;
        if (t->rotate != 0 && t->rotate != 1) return -1;
        if (t->rotate) {
            if (!(isfinite(t->ra0) && isfinite(t->dec0) && isfinite(t->ra1) && isfinite(t->dec1))) return -1;
            ora_frame f;
            ora_make_frame(t, &f);
            if (!(f.R[8] > 0.0)) return -1;     /* the stacking position must face the phase centre */
        } else if (!(t->l * t->l + t->m * t->m < 1.0)) return -1;
    }
    return 0;
}

/* The stack over rest channels [jlo, jhi).  Outputs are dense over that slab:
 * S [jhi-jlo][nv][nu][2], W, A [jhi-jlo][nv][nu], N likewise (uint64).  Any of
 * them may be NULL.  stats (7 x uint64, may be NULL) classifies every sample of
 * every target, whatever the slab:
 *   [0] samples  [1] flagged  [2] bad weight  [3] outside uv  [4] outside band
 *   [5] used     [6] contributions (pairs (sample, j) over all j).
 * Classification order: outside band (J_k empty) -> outside uv -> flagged ->
 * weight not finite or not > 0 -> used. */
int ora_stack(const ora_grid* g, int32_t ntgt, const ora_target* tg, int32_t jlo, int32_t jhi,
              double* S, double* W, double* A, uint64_t* N, uint64_t* stats, int nthreads) {
    if (ora_check(g, ntgt, tg)) return -1;
    if (jlo < 0 || jhi > g->nchan || jlo > jhi) return -1;
    size_t plane = (size_t)g->nu * g->nv;
    size_t ncell = plane * (size_t)(jhi - jlo);
    if (S) memset(S, 0, sizeof(double) * 2 * ncell);
    if (W) memset(W, 0, sizeof(double) * ncell);
    if (A) memset(A, 0, sizeof(double) * ncell);
    if (N) memset(N, 0, sizeof(uint64_t) * ncell);
    if (stats) memset(stats, 0, sizeof(uint64_t) * 7);

    ora_table* tabs = (ora_table*)calloc(ntgt > 0 ? ntgt : 1, sizeof(ora_table));
    if (!tabs) return -3;
    int rc = 0;
    for (int32_t i = 0; i < ntgt && !rc; ++i) rc = ora_build_table(g, &tg[i], &tabs[i]);
    if (rc) { for (int32_t i = 0; i < ntgt; ++i) ora_free_table(&tabs[i]); free(tabs); return rc; }

    int nth = 1;
#ifdef _OPENMP
    nth = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    if (nth > jhi - jlo) nth = jhi - jlo > 0 ? jhi - jlo : 1;

#ifdef _OPENMP
#pragma omp parallel num_threads(nth)
#endif
    {
        int th = 0;
#ifdef _OPENMP
        th = omp_get_thread_num();
#endif
        /* this thread's rest-channel slab */
        int32_t span = jhi - jlo;
        int32_t ja = jlo + (int32_t)((int64_t)span * th / nth);
        int32_t jb = jlo + (int32_t)((int64_t)span * (th + 1) / nth);
        for (int32_t i = 0; i < ntgt; ++i) {
            const ora_target* t = &tg[i];
            const ora_table* tb = &tabs[i];
            ora_frame fr;
            ora_make_frame(t, &fr);
            for (int64_t r = 0; r < t->nrow; ++r) {
                const double* uvw = t->uvw + 3 * r;
                double ur[3];
                ora_rot(&fr, uvw, ur);
                for (int32_t k = t->kbeg; k < t->kend; ++k) {
                    int32_t q0 = tb->start[k], q1 = tb->start[k + 1], q;
                    int mine = 0;
                    for (q = q0; q < q1; ++q) mine |= (tb->j[q] >= ja && tb->j[q] < jb);
                    if (!mine) continue;
                    int64_t iu, iv;
                    if (!ora_cell(g, ur, tb->a[k], &iu, &iv)) continue;
                    double pc, ps;
                    ora_phasor(uvw, tb->a[k], fr.l, fr.m, fr.nm1, &pc, &ps);
                    for (int32_t p = 0; p < t->npol; ++p) {
                        size_t e = ora_elem(t, r, k, p);
                        if (t->flag && t->flag[e]) continue;
                        double wt = ora_weight(t, r, k, p);
                        if (!(wt > 0.0 && isfinite(wt))) continue;
                        double vr = (double)t->vis[2 * e], vi = (double)t->vis[2 * e + 1];
                        double xr = vr * pc - vi * ps;      /* V' = V * (pc + i ps) */
                        double xi = vr * ps + vi * pc;
                        double mag = sqrt(xr * xr + xi * xi);
                        for (q = q0; q < q1; ++q) {
                            int32_t j = tb->j[q];
                            if (j < ja || j >= jb) continue;
                            double wf = wt * tb->f[q];
                            size_t c = (size_t)(j - jlo) * plane + (size_t)iv * g->nu + (size_t)iu;
                            if (S) { S[2 * c] += wf * xr; S[2 * c + 1] += wf * xi; }
                            if (W) W[c] += wf;
                            if (A) A[c] += wf * mag;
                            if (N) N[c] += 1;
                        }
                    }
                }
            }
        }
    }

    if (stats) {
        for (int32_t i = 0; i < ntgt; ++i) {
            const ora_target* t = &tg[i];
            const ora_table* tb = &tabs[i];
            ora_frame fr;
            ora_make_frame(t, &fr);
            for (int64_t r = 0; r < t->nrow; ++r) {
                double ur[3];
                ora_rot(&fr, t->uvw + 3 * r, ur);
                for (int32_t k = t->kbeg; k < t->kend; ++k) {
                    int32_t nj = tb->start[k + 1] - tb->start[k];
                    int64_t iu, iv;
                    int inside = nj > 0 ? ora_cell(g, ur, tb->a[k], &iu, &iv) : 0;
                    for (int32_t p = 0; p < t->npol; ++p) {
                        size_t e = ora_elem(t, r, k, p);
                        stats[0]++;
                        if (nj == 0) { stats[4]++; continue; }
                        if (!inside) { stats[3]++; continue; }
                        if (t->flag && t->flag[e]) { stats[1]++; continue; }
                        double wt = ora_weight(t, r, k, p);
                        if (!(wt > 0.0 && isfinite(wt))) { stats[2]++; continue; }
                        stats[5]++;
                        stats[6] += (uint64_t)nj;
                    }
                }
            }
        }
    }
    for (int32_t i = 0; i < ntgt; ++i) ora_free_table(&tabs[i]);
    free(tabs);
    return 0;
}

/* Per (row, channel) indices of one target for channels [kbeg, kend): the uv cell
 * (iu, iv) as computed before the grid-bounds test, and the first rest channel and
 * size of J_k (j0 = -1, nj = 0 when J_k is empty). */
int ora_indices(const ora_grid* g, const ora_target* t, int64_t* iu, int64_t* iv, int32_t* j0,
                int32_t* nj) {
    if (ora_check(g, 1, t)) return -1;
    ora_table tb;
    int rc = ora_build_table(g, t, &tb);
    if (rc) { ora_free_table(&tb); return rc; }
    int32_t nk = t->kend - t->kbeg;
    ora_frame fr;
    ora_make_frame(t, &fr);
    for (int64_t r = 0; r < t->nrow; ++r) {
        double ur[3];
        ora_rot(&fr, t->uvw + 3 * r, ur);
        for (int32_t k = t->kbeg; k < t->kend; ++k) {
            size_t e = (size_t)r * nk + (k - t->kbeg);
            int64_t a, b;
            ora_cell(g, ur, tb.a[k], &a, &b);
            iu[e] = a;
            iv[e] = b;
            int32_t n = tb.start[k + 1] - tb.start[k];
            nj[e] = n;
            j0[e] = n ? tb.j[tb.start[k]] : -1;
        }
    }
    ora_free_table(&tb);
    return 0;
}

/* The rotated visibilities V' = V exp(+2 pi i t) of every sample (Eq. 2), regardless
 * of flags and weights: out [nrow][kend-kbeg][npol][2]. */
int ora_rotate(const ora_target* t, double* out) {
    if (t->nchan < 1 || t->kbeg < 0 || t->kend > t->nchan || t->kbeg > t->kend) return -1;
    ora_frame fr;
    ora_make_frame(t, &fr);
    int32_t nk = t->kend - t->kbeg;
    for (int64_t r = 0; r < t->nrow; ++r) {
        for (int32_t k = t->kbeg; k < t->kend; ++k) {
            double pc, ps;
            ora_phasor(t->uvw + 3 * r, t->chan_freq[k] / ORA_C, fr.l, fr.m, fr.nm1, &pc, &ps);
            for (int32_t p = 0; p < t->npol; ++p) {
                size_t e = ((size_t)r * nk + (k - t->kbeg)) * t->npol + p;
                size_t d = ora_elem(t, r, k, p);
                double vr = (double)t->vis[2 * d], vi = (double)t->vis[2 * d + 1];
                out[2 * e] = vr * pc - vi * ps;
                out[2 * e + 1] = vr * ps + vi * pc;
            }
        }
    }
    return 0;
}

/* The channel table of one target: a_k, W_k, rest edges, and J_k as CSR
 * (start[nchan+1], j[], f[]).  Call with j == NULL first to get the pair count in
 * *npairs, then again with arrays of that size. */
int ora_channel_table(const ora_grid* g, const ora_target* t, double* a, double* width, double* lo,
                      double* hi, int32_t* start, int32_t* j, double* f, int32_t* npairs) {
    if (ora_check(g, 1, t)) return -1;
    ora_table tb;
    int rc = ora_build_table(g, t, &tb);
    if (rc) { ora_free_table(&tb); return rc; }
    int32_t n = tb.nchan, np = tb.start[n];
    if (j && f && *npairs >= np) {
        memcpy(j, tb.j, sizeof(int32_t) * np);
        memcpy(f, tb.f, sizeof(double) * np);
    }
    if (a) memcpy(a, tb.a, sizeof(double) * n);
    if (width) memcpy(width, tb.width, sizeof(double) * n);
    if (lo) memcpy(lo, tb.lo, sizeof(double) * n);
    if (hi) memcpy(hi, tb.hi, sizeof(double) * n);
    if (start) memcpy(start, tb.start, sizeof(int32_t) * (n + 1));
    *npairs = np;
    ora_free_table(&tb);
    return 0;
}

/* The paper's common output grid (Sec. 3.1): the rest channel width is the widest
 * rest-frame input channel of all targets, Delta nu_new = max_i Delta nu_rf,i, and the
 * nchan_out channels are centred on central_freq. */
int ora_plan_spectral_grid(int32_t n, const double* const* chan_freq, const double* const* chan_width,
                           const int32_t* nchan, const double* z, double central_freq,
                           int32_t nchan_out, double* freq_lo, double* dfreq) {
    if (n < 1 || nchan_out < 1) return -1;
    double wmax = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        if (nchan[i] < 1 || (nchan[i] == 1 && !(chan_width && chan_width[i]))) return -1;
        for (int32_t k = 0; k < nchan[i]; ++k) {
            double W = ora_width(chan_freq[i], chan_width ? chan_width[i] : NULL, nchan[i], k);
            double Wr = W * (1.0 + z[i]);
            if (Wr > wmax) wmax = Wr;
        }
    }
    if (!(wmax > 0.0)) return -1;
    *dfreq = wmax;
    *freq_lo = central_freq - 0.5 * (double)nchan_out * wmax;
    return 0;
}

/* ------------------------------------------------------------------- rebinned rows */

/* The lower edge of one target's own output window (Sec. 3.1): nout channels of the common
 * rest width dfreq, centred on central_freq.  When that window does not fit inside the
 * target's rest-frame band [lo, hi] (the outermost rest edges of its channels), it moves to
 * the nearest band edge: its upper edge down to hi if it overhangs there, and then, if it
 * still starts below lo (which a window wider than the band does), its lower edge up to
 * lo. */
int ora_rebin_window(const ora_target* t, double central_freq, double dfreq, int32_t nout, double* freq_lo) {
    if (!t || t->nchan < 1 || nout < 1 || !(dfreq > 0.0) || !isfinite(dfreq) || !isfinite(central_freq))
        return -1;
    if (t->nchan == 1 && !t->chan_width) return -1;
    double opz = 1.0 + t->z;
    double lo = INFINITY, hi = -INFINITY;
    for (int32_t k = 0; k < t->nchan; ++k) {
        double W = ora_width(t->chan_freq, t->chan_width, t->nchan, k);
        lo = fmin(lo, (t->chan_freq[k] - 0.5 * W) * opz);
        hi = fmax(hi, (t->chan_freq[k] + 0.5 * W) * opz);
    }
    double wid = (double)nout * dfreq;
    double s = central_freq - 0.5 * wid;
    if (s + wid > hi) s = hi - wid;
    if (s < lo) s = lo;
    *freq_lo = s;
    return 0;
}

/* One target's rows rebinned onto its own window [freq_lo + j dfreq, freq_lo + (j+1) dfreq),
 * j < nout, row by row (the product of the paper's per-row kernel, Sec. 3.2):
 *   out[r][j][p] = sum_k f_kj V'(r,k,p) / sum_k f_kj,
 * the sums over the input channels k whose Eq. 4 overlap f_kj with channel j is above the
 * sliver threshold and whose sample (r, k, p) is not flagged; V' is the Eq. 2-rotated
 * visibility, in double.  Where no such channel exists the output is 0 and flagged.
 * wsum[r][j][p] = sum_k f_kj (0 where flagged).  uvw_out[r] = R uvw[r] / (1 + z), the
 * rest-frame baseline of Eq. 1 (R the identity unless the target asks for the rotation).  Visibility
 * weights do not enter Eq. 3.  The data arrays must hold all channels. */
int ora_rebin_rows(const ora_target* t, double freq_lo, double dfreq, int32_t nout, double* out,
                   uint8_t* oflag, double* wsum, double* uvw_out) {
    ora_grid g;
    g.nu = 1; g.nv = 1; g.nchan = nout; g.du = 1.0; g.dv = 1.0;
    g.freq_lo = freq_lo; g.dfreq = dfreq; g.flags = 0;
    if (ora_check(&g, 1, t)) return -1;
    if (t->kbeg != 0 || t->kend != t->nchan) return -1;
    ora_table tb;
    int rc = ora_build_table(&g, t, &tb);
    if (rc) { ora_free_table(&tb); return rc; }
    const int32_t np = t->npol, nk = t->nchan;
    const double opz = 1.0 + t->z;
    ora_frame fr;
    ora_make_frame(t, &fr);
    double* num = (double*)malloc(sizeof(double) * 2 * (size_t)nout * np);
    double* den = (double*)malloc(sizeof(double) * (size_t)nout * np);
    if (!num || !den) { free(num); free(den); ora_free_table(&tb); return -3; }
    for (int64_t r = 0; r < t->nrow; ++r) {
        memset(num, 0, sizeof(double) * 2 * (size_t)nout * np);
        memset(den, 0, sizeof(double) * (size_t)nout * np);
        for (int32_t k = 0; k < nk; ++k) {
            double pc, ps;
            ora_phasor(t->uvw + 3 * r, tb.a[k], fr.l, fr.m, fr.nm1, &pc, &ps);
            for (int32_t q = tb.start[k]; q < tb.start[k + 1]; ++q) {
                const int32_t j = tb.j[q];
                const double f = tb.f[q];
                for (int32_t p = 0; p < np; ++p) {
                    size_t e = ((size_t)r * nk + k) * np + p;
                    if (t->flag && t->flag[e]) continue;
                    double vr = (double)t->vis[2 * e], vi = (double)t->vis[2 * e + 1];
                    num[2 * ((size_t)j * np + p)] += f * (vr * pc - vi * ps);
                    num[2 * ((size_t)j * np + p) + 1] += f * (vr * ps + vi * pc);
                    den[(size_t)j * np + p] += f;
                }
            }
        }
        for (int32_t j = 0; j < nout; ++j)
            for (int32_t p = 0; p < np; ++p) {
                size_t o = ((size_t)r * nout + j) * np + p;
                double d = den[(size_t)j * np + p];
                out[2 * o] = d > 0.0 ? num[2 * ((size_t)j * np + p)] / d : 0.0;
                out[2 * o + 1] = d > 0.0 ? num[2 * ((size_t)j * np + p) + 1] / d : 0.0;
                if (oflag) oflag[o] = d > 0.0 ? 0 : 1;
                if (wsum) wsum[o] = d;
            }
        if (uvw_out) {
            double ur[3];
            ora_rot(&fr, t->uvw + 3 * r, ur);
            for (int i = 0; i < 3; ++i) uvw_out[3 * r + i] = ur[i] / opz;
        }
    }
    free(num);
    free(den);
    ora_free_table(&tb);
    return 0;
}


/* Eq. 1's rotation of one target as the oracle uses it: R (row-major 3 x 3) and the
 * direction cosines (l, m) with n - 1 (for tests). */
int ora_frame_matrix(const ora_target* t, double* R, double* lm_nm1) {
    if (!t || (t->rotate != 0 && t->rotate != 1)) return -1;
    ora_frame f;
    ora_make_frame(t, &f);
    for (int i = 0; i < 9; ++i) R[i] = f.R[i];
    lm_nm1[0] = f.l;
    lm_nm1[1] = f.m;
    lm_nm1[2] = f.nm1;
    return 0;
}

/* ------------------------------------------------------------------- dirty image */

/* The dirty image of one rest channel of a stacked grid by direct Fourier inversion (the
 * imaging the paper's outlook, Sec. 3.4, would do with an FFT on the stacked product):
 *   I(q, p) = Re sum_{iv, iu} S[iv][iu] exp(+2 pi i (u x_p + v y_q)) / W_total,
 * with u = (iu - nu/2) du, v = (iv - nv/2) dv, x_p = (p - nu/2) / (nu du) and
 * y_q = (q - nv/2) / (nv dv): the phase is 2 pi ((iu - nu/2)(p - nu/2) / nu +
 * (iv - nv/2)(q - nv/2) / nv), independent of du and dv; its integer numerators are
 * reduced modulo nu and nv (an exact identity) before the trigonometry.  W_total is the
 * channel's summed weight; the image is 0 where it is 0.  The gridded data hold each
 * measured baseline once, so the real part is the dirty image of a real sky.
 * S [nv][nu][2], W [nv][nu]. */
static double ora_pixel(int32_t nu, int32_t nv, const double* S, double wt, int32_t q, int32_t p) {
    if (!(wt > 0.0)) return 0.0;
    const int64_t cu = nu / 2, cv = nv / 2;
    double acc = 0.0;
    for (int32_t iv = 0; iv < nv; ++iv) {
        const int64_t av = (((int64_t)(iv - cv) * (q - cv)) % nv + nv) % nv;
        for (int32_t iu = 0; iu < nu; ++iu) {
            const double sr = S[2 * ((size_t)iv * nu + iu)], si = S[2 * ((size_t)iv * nu + iu) + 1];
            if (sr == 0.0 && si == 0.0) continue;
            const int64_t au = (((int64_t)(iu - cu) * (p - cu)) % nu + nu) % nu;
            const double ph = 2.0 * ORA_PI * ((double)au / (double)nu + (double)av / (double)nv);
            acc += sr * cos(ph) - si * sin(ph);
        }
    }
    return acc / wt;
}

/* Every pixel of every channel: S [nchan][nv][nu][2], W [nchan][nv][nu]; img and beam
 * [nchan][nv][nu] (either may be NULL; the beam is the same inversion of W). */
int ora_image(int32_t nu, int32_t nv, int32_t nchan, const double* S, const double* W, double* img, double* beam) {
    if (nu < 1 || nv < 1 || nchan < 0) return -1;
    const size_t plane = (size_t)nu * nv;
    double* wre = (double*)malloc(sizeof(double) * 2 * plane);
    if (!wre) return -3;
    for (int32_t j = 0; j < nchan; ++j) {
        const double* Sj = S + 2 * plane * j;
        const double* Wj = W + plane * j;
        double wt = 0.0;
        for (size_t c = 0; c < plane; ++c) wt += Wj[c];
        for (size_t c = 0; c < plane; ++c) { wre[2 * c] = Wj[c]; wre[2 * c + 1] = 0.0; }
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int32_t q = 0; q < nv; ++q)
            for (int32_t p = 0; p < nu; ++p) {
                if (img) img[plane * j + (size_t)q * nu + p] = ora_pixel(nu, nv, Sj, wt, q, p);
                if (beam) beam[plane * j + (size_t)q * nu + p] = ora_pixel(nu, nv, wre, wt, q, p);
            }
    }
    free(wre);
    return 0;
}

/* Selected pixels (q[i], p[i]) of one channel (S [nv][nu][2], W [nv][nu]). */
int ora_image_pixels(int32_t nu, int32_t nv, const double* S, const double* W, int32_t n, const int32_t* q,
                     const int32_t* p, double* out) {
    if (nu < 1 || nv < 1 || n < 0) return -1;
    double wt = 0.0;
    for (size_t c = 0; c < (size_t)nu * nv; ++c) wt += W[c];
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int32_t i = 0; i < n; ++i) out[i] = ora_pixel(nu, nv, S, wt, q[i], p[i]);
    return 0;
}
