// Host planning: validation and the per-target rest-frame channel table.
//
// Compiled with -ffp-contract=off and without fast-math: the rest edges, output edges and
// overlap fractions follow the definition's FP64 operation sequence exactly, so the
// rest-channel indices equal those of any other exact implementation of it.
#include "vista_plan.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>

namespace vista {

namespace {
constexpr double kSliver = 1e-9;  // overlap fractions at or below this are dropped

std::string fmt(const char* f, double a = 0, double b = 0) {
    char buf[256];
    snprintf(buf, sizeof(buf), f, a, b);
    return buf;
}
}  // namespace

double channel_width(const double* f, const double* w, int32_t n, int32_t k) {
    if (w) return w[k];
    if (n < 2) return NAN;
    if (k == 0) return fabs(f[1] - f[0]);
    if (k == n - 1) return fabs(f[n - 1] - f[n - 2]);
    return fabs(f[k + 1] - f[k - 1]) / 2.0;
}

Frame make_frame(const vista_target* t) {
    Frame f;
    f.rotate = t->rotate_uvw;
    if (t->rotate_uvw) {
        // uvw axes (east, north, towards) of the two centres in equatorial coordinates
        auto axes = [](double ra, double dec, double ax[3][3]) {
            ax[0][0] = -sin(ra);            ax[0][1] = cos(ra);             ax[0][2] = 0.0;
            ax[1][0] = -sin(dec) * cos(ra); ax[1][1] = -sin(dec) * sin(ra); ax[1][2] = cos(dec);
            ax[2][0] = cos(dec) * cos(ra);  ax[2][1] = cos(dec) * sin(ra);  ax[2][2] = sin(dec);
        };
        double a0[3][3], a1[3][3];
        axes(t->ra0, t->dec0, a0);
        axes(t->ra1, t->dec1, a1);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                f.R[3 * i + j] = a1[i][0] * a0[j][0] + a1[i][1] * a0[j][1] + a1[i][2] * a0[j][2];
        f.l = f.R[6];
        f.m = f.R[7];
    } else {
        f.l = t->l;
        f.m = t->m;
    }
    return f;
}

bool check_grid(const vista_grid_desc* g, std::string* why) {
    if (!g) { *why = "grid descriptor is NULL"; return false; }
    if (g->nu < 1 || g->nv < 1 || g->nu > 65535 || g->nv > 65535) {
        *why = fmt("grid nu, nv must be in 1..65535 (got %g, %g)", g->nu, g->nv);
        return false;
    }
    if (g->nchan < 1 || g->nchan >= (int32_t)kJMask) { *why = "grid nchan must be in 1..16777214"; return false; }
    if (!(g->du > 0 && isfinite(g->du) && g->dv > 0 && isfinite(g->dv))) {
        *why = fmt("grid du, dv must be finite and > 0 (got %g, %g)", g->du, g->dv);
        return false;
    }
    if (!(g->dfreq > 0 && isfinite(g->dfreq))) { *why = "grid dfreq must be finite and > 0"; return false; }
    if (!isfinite(g->freq_lo)) { *why = "grid freq_lo must be finite"; return false; }
    if (g->flags & ~(uint32_t)(VISTA_F_KAHAN | VISTA_F_DETERMINISTIC | VISTA_F_SPECTRAL_NEAREST |
                               VISTA_F_PHASE_FP32 | VISTA_F_PLAIN_FP32)) {
        *why = "unknown grid flag bits";
        return false;
    }
    if ((g->flags & VISTA_F_PLAIN_FP32) && (g->flags & (VISTA_F_KAHAN | VISTA_F_DETERMINISTIC))) {
        *why = "VISTA_F_PLAIN_FP32 (uncompensated FP32 tiles) excludes VISTA_F_KAHAN and VISTA_F_DETERMINISTIC";
        return false;
    }
    if ((double)g->nu * g->nv * g->nchan > 4.0e11) { *why = "grid has too many cells"; return false; }
    return true;
}

bool check_target(const vista_grid_desc* g, const vista_target* t, std::string* why) {
    if (!t) { *why = "target is NULL"; return false; }
    if (t->nrow < 0) { *why = "target nrow must be >= 0"; return false; }
    if (t->nrow > 0x7fffffffLL) { *why = "target nrow must be < 2^31"; return false; }
    if (t->nchan < 1 || t->nchan > 65535) { *why = "target nchan must be in 1..65535"; return false; }
    if (t->npol != 1 && t->npol != 2 && t->npol != 4) { *why = "target npol must be 1, 2 or 4"; return false; }
    if (t->mem != VISTA_MEM_HOST && t->mem != VISTA_MEM_HOST_PINNED && t->mem != VISTA_MEM_DEVICE) {
        *why = "target mem must be a VISTA_MEM_* value";
        return false;
    }
    if (t->weight_per_chan != 0 && t->weight_per_chan != 1) { *why = "weight_per_chan must be 0 or 1"; return false; }
    if (!t->chan_freq) { *why = "chan_freq is NULL"; return false; }
    if (t->nrow > 0 && (!t->uvw || !t->vis || !t->weight)) { *why = "uvw, vis and weight are required"; return false; }
    if (t->nchan == 1 && !t->chan_width) { *why = "nchan == 1 needs chan_width"; return false; }
    if (!(t->z > -1.0 && isfinite(t->z))) { *why = fmt("z must be finite and > -1 (got %g)", t->z); return false; }
    if (t->rotate_uvw != 0 && t->rotate_uvw != 1) { *why = "rotate_uvw must be 0 or 1"; return false; }
    if (t->rotate_uvw) {
        if (!(isfinite(t->ra0) && isfinite(t->dec0) && isfinite(t->ra1) && isfinite(t->dec1))) {
            *why = "ra0, dec0, ra1, dec1 must be finite";
            return false;
        }
        if (!(make_frame(t).R[8] > 0.0)) {
            *why = "the stacking position must lie in the phase centre's front hemisphere";
            return false;
        }
    } else if (!(isfinite(t->l) && isfinite(t->m) && t->l * t->l + t->m * t->m < 1.0)) {
        *why = fmt("need l*l + m*m < 1 (got l=%g, m=%g)", t->l, t->m);
        return false;
    }
    double dir = 0;
    for (int32_t k = 0; k < t->nchan; ++k) {
        double f = t->chan_freq[k];
        if (!(f > 0 && isfinite(f))) { *why = fmt("chan_freq[%g] must be finite and > 0", k); return false; }
        if (t->chan_width && !(t->chan_width[k] > 0 && isfinite(t->chan_width[k]))) {
            *why = fmt("chan_width[%g] must be finite and > 0", k);
            return false;
        }
        if (k > 0) {
            double d = f - t->chan_freq[k - 1];
            if (d == 0 || (dir != 0 && (d > 0) != (dir > 0))) {
                *why = fmt("chan_freq must be strictly monotonic (channel %g)", k);
                return false;
            }
            dir = d;
        }
    }
    // vector loads: a (row, channel) of complex64 x npol is read as 8, 16 or 2x16 bytes,
    // its flags as 1, 2 or 4 bytes
    if (t->nrow > 0) {
        size_t va = t->npol == 1 ? 8 : 16;
        if (((uintptr_t)t->vis % va) != 0) { *why = "vis must be 16-byte aligned (8 for npol == 1)"; return false; }
        if (t->flag && ((uintptr_t)t->flag % (size_t)t->npol) != 0) {
            *why = "flag must be aligned to npol bytes";
            return false;
        }
        if (((uintptr_t)t->uvw % 8) != 0 || ((uintptr_t)t->weight % 4) != 0) {
            *why = "uvw must be 8-byte and weight 4-byte aligned";
            return false;
        }
    }
    (void)g;
    return true;
}

ChannelPlan plan_target(const vista_grid_desc* g, const vista_target* t) {
    ChannelPlan p;
    const int32_t n = t->nchan;
    const double opz = 1.0 + t->z;
    p.frame = make_frame(t);
    const double lm2 = p.frame.l * p.frame.l + p.frame.m * p.frame.m;
    p.nm1 = -lm2 / (1.0 + sqrt(1.0 - lm2));
    p.chan.resize(n);
    p.f1.assign(n, 0.f);
    p.foff.assign(n, 0);
    p.j0.assign(n, -1);
    p.nj.assign(n, 0);
    p.inband.assign(n + 1, 0);
    for (int32_t k = 0; k < n; ++k) {
        struct { int32_t j0, nj; float f0, f1; } c = {-1, 0, 0.f, 0.f};
        p.foff[k] = (int32_t)p.fval.size();
        if (g->flags & VISTA_F_SPECTRAL_NEAREST) {
            double x = floor((t->chan_freq[k] * opz - g->freq_lo) / g->dfreq);
            if (x >= 0.0 && x < (double)g->nchan) {
                c.j0 = (int32_t)x;
                c.nj = 1;
                c.f0 = 1.0f;
                p.fval.push_back(1.0f);
            }
        } else {
            double W = channel_width(t->chan_freq, t->chan_width, n, k);
            double lo = (t->chan_freq[k] - 0.5 * W) * opz;
            double hi = (t->chan_freq[k] + 0.5 * W) * opz;
            double Wr = W * opz;
            // candidate rest channels around [lo, hi), widened; each tested exactly
            double x0 = floor((lo - g->freq_lo) / g->dfreq) - 2.0;
            double x1 = floor((hi - g->freq_lo) / g->dfreq) + 2.0;
            int32_t ja = (int32_t)std::max(0.0, std::min(x0, (double)g->nchan));
            int32_t jb = (int32_t)std::max(-1.0, std::min(x1, (double)g->nchan - 1));
            for (int32_t j = ja; j <= jb; ++j) {
                double e0 = g->freq_lo + (double)j * g->dfreq;
                double e1 = g->freq_lo + (double)(j + 1) * g->dfreq;
                double ov = fmin(hi, e1) - fmax(lo, e0);
                double f = ov / Wr;
                if (f > kSliver) {
                    if (c.nj == 0) c.j0 = j;
                    if (c.nj == 0) c.f0 = (float)f;
                    if (c.nj == 1) c.f1 = (float)f;
                    c.nj++;
                    p.fval.push_back((float)f);
                }
            }
        }
        p.inband[k + 1] = p.inband[k] + (c.nj > 0 ? 1 : 0);
        p.j0[k] = c.j0;
        p.nj[k] = c.nj;
        p.f1[k] = c.f1;
        DevChan& d = p.chan[k];
        d.a = t->chan_freq[k] / kC;
        d.jn = c.nj > 0 ? ((uint32_t)c.j0 | ((uint32_t)std::min(c.nj, kMaxNj) << 24)) : kJMask;
        d.f0 = c.f0;
    }
    p.n_inband = p.inband[n];
    p.kin_lo = n;
    p.kin_hi = 0;
    for (int32_t k = 0; k < n; ++k) {
        if (p.nj[k] > 0) {
            p.kin_lo = std::min(p.kin_lo, k);
            p.kin_hi = std::max(p.kin_hi, k + 1);
        }
    }
    if (p.kin_lo >= p.kin_hi) { p.kin_lo = 0; p.kin_hi = 0; }
    // Lanes `nphase` channels apart never reach the same rest channel: two channels that
    // share rest channel j are at most (last - first channel reaching j) apart.
    std::vector<int32_t> kmin(g->nchan, INT32_MAX), kmax(g->nchan, -1);
    for (int32_t k = 0; k < n; ++k) {
        for (int32_t q = 0; q < p.nj[k]; ++q) {
            int32_t j = p.j0[k] + q;
            kmin[j] = std::min(kmin[j], k);
            kmax[j] = std::max(kmax[j], k);
        }
    }
    int32_t span = 0, reached = 0;
    for (int32_t j = 0; j < g->nchan; ++j)
        if (kmax[j] >= 0) {
            span = std::max(span, kmax[j] - kmin[j]);
            ++reached;
        }
    p.chan_per_rest = reached > 0 ? (double)p.n_inband / (double)reached : 0.0;
    p.nphase = std::min(64, span + 1);
    if (p.nphase < 1) p.nphase = 1;
    return p;
}

double rebin_window(const vista_target* t, double central_freq, double dfreq, int32_t nout) {
    const double opz = 1.0 + t->z;
    double lo = INFINITY, hi = -INFINITY;
    for (int32_t k = 0; k < t->nchan; ++k) {
        const double W = channel_width(t->chan_freq, t->chan_width, t->nchan, k);
        lo = fmin(lo, (t->chan_freq[k] - 0.5 * W) * opz);
        hi = fmax(hi, (t->chan_freq[k] + 0.5 * W) * opz);
    }
    const double wid = (double)nout * dfreq;
    double s = central_freq - 0.5 * wid;
    if (s + wid > hi) s = hi - wid;
    if (s < lo) s = lo;
    return s;
}

RebinPlan plan_rebin(const vista_target* t, double freq_lo, double dfreq, int32_t nout) {
    vista_grid_desc g;
    memset(&g, 0, sizeof(g));
    g.nu = 1; g.nv = 1; g.du = 1.0; g.dv = 1.0;
    g.nchan = nout; g.freq_lo = freq_lo; g.dfreq = dfreq; g.flags = 0;
    const ChannelPlan p = plan_target(&g, t);
    RebinPlan r;
    r.nm1 = p.nm1;
    r.frame = p.frame;
    r.a.resize(t->nchan);
    for (int32_t k = 0; k < t->nchan; ++k) r.a[k] = p.chan[k].a;
    r.jstart.assign((size_t)nout + 1, 0);
    for (int32_t k = 0; k < t->nchan; ++k)
        for (int32_t q = 0; q < p.nj[k]; ++q) r.jstart[p.j0[k] + q + 1]++;
    for (int32_t j = 0; j < nout; ++j) r.jstart[j + 1] += r.jstart[j];
    r.ek.resize(r.jstart[nout]);
    r.ef.resize(r.jstart[nout]);
    std::vector<int32_t> fill(r.jstart.begin(), r.jstart.end() - 1);
    for (int32_t k = 0; k < t->nchan; ++k)
        for (int32_t q = 0; q < p.nj[k]; ++q) {
            const int32_t j = p.j0[k] + q, e = fill[j]++;
            r.ek[e] = k;
            r.ef[e] = p.fval[p.foff[k] + q];
        }
    return r;
}

bool check_plan(const ChannelPlan& p, std::string* why) {
    for (size_t k = 0; k < p.nj.size(); ++k) {
        if (p.nj[k] > kMaxNj) {
            *why = "a channel overlaps more than 255 rest channels (rest grid too fine for the data)";
            return false;
        }
    }
    return true;
}

std::vector<int32_t> block_ranges(const ChannelPlan& p, int32_t nchan_grid, int32_t jsub) {
    int32_t nb = (nchan_grid + jsub - 1) / jsub;
    std::vector<int32_t> out(2 * (size_t)nb, 0);
    std::vector<int32_t> lo(nb, INT32_MAX), hi(nb, INT32_MIN);
    for (int32_t k = 0; k < (int32_t)p.chan.size(); ++k) {
        for (int32_t q = 0; q < p.nj[k]; ++q) {
            int32_t b = (p.j0[k] + q) / jsub;
            lo[b] = std::min(lo[b], k);
            hi[b] = std::max(hi[b], k + 1);
        }
    }
    for (int32_t b = 0; b < nb; ++b) {
        if (lo[b] < hi[b]) { out[2 * b] = lo[b]; out[2 * b + 1] = hi[b]; }
    }
    return out;
}

}  // namespace vista
