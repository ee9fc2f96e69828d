// Host planning of one target (rest-frame channel table) and argument validation.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "vista.h"
#include "vista_internal.h"

namespace vista {

// Eq. 1's rotation of a target: R (row-major) from the phase centre's uvw axes to the
// stacking position's, and the direction cosines (l, m) the Eq. 2 shift uses (the given
// ones without the rotation, R then the identity).
struct Frame {
    int32_t rotate = 0;
    double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    double l = 0.0, m = 0.0;
};
Frame make_frame(const vista_target* t);

// Per-target rest-frame plan (Sec. 3.1 and Eq. 3-4), computed in FP64 on the host.
struct ChannelPlan {
    std::vector<DevChan> chan;     // [nchan]
    std::vector<float> f1;         // [nchan] second overlap fraction (0 if nj < 2)
    std::vector<int32_t> foff;     // [nchan] offset of the channel's fractions in fval
    std::vector<float> fval;       // overlap fractions of every channel, in order
    std::vector<int32_t> j0, nj;   // [nchan] unpacked J_k ranges (host use)
    std::vector<int32_t> inband;   // [nchan+1] prefix count of channels with nj > 0
    int32_t kin_lo = 0, kin_hi = 0;  // hull of channels with nj > 0
    int32_t nphase = 1;            // channel distance with disjoint rest-channel sets
    int64_t n_inband = 0;          // channels with nj > 0
    double chan_per_rest = 0.0;    // in-band channels per rest channel they reach
    double nm1 = 0.0;              // n - 1 for (l, m)
    Frame frame;                   // Eq. 1's rotation and the (l, m) in use
};

// Validation; on failure returns false and fills *why.
bool check_grid(const vista_grid_desc* g, std::string* why);
bool check_target(const vista_grid_desc* g, const vista_target* t, std::string* why);
// Channel-table limits of the packed device format (J_k sizes up to kMaxNj); false with
// *why when the target's overlap sets do not fit.
bool check_plan(const ChannelPlan& p, std::string* why);

// Build the plan of target t on grid g.
ChannelPlan plan_target(const vista_grid_desc* g, const vista_target* t);

// k ranges [lo, hi) of the channels reaching each rest-channel block of size jsub:
// out[2b], out[2b+1]; empty blocks get lo = hi = 0.
std::vector<int32_t> block_ranges(const ChannelPlan& p, int32_t nchan_grid, int32_t jsub);

// Input channel width W_k (Eq. 4's Delta nu_k): given width, else centred difference.
double channel_width(const double* f, const double* w, int32_t n, int32_t k);

// Lower edge of target t's own output window (Sec. 3.1): nout channels of width dfreq
// centred on central_freq, moved to the nearest edge of the target's rest-frame band when
// it does not fit (upper edge first, then lower edge).
double rebin_window(const vista_target* t, double central_freq, double dfreq, int32_t nout);

// Per-output-channel lists of the Eq. 4 fractions of target t on its window: for output
// channel j, entries [jstart[j], jstart[j+1]) of (ek, ef) are the input channels (in
// ascending order) and their fractions.
struct RebinPlan {
    std::vector<double> a;         // [nchan] nu_k / c
    std::vector<int32_t> jstart;   // [nout+1]
    std::vector<int32_t> ek;
    std::vector<float> ef;
    double nm1 = 0.0;
    Frame frame;
};
RebinPlan plan_rebin(const vista_target* t, double freq_lo, double dfreq, int32_t nout);

}  // namespace vista
