// Internal types shared by the host runtime (vista_runtime.cpp) and the gfx950 kernels
// (vista_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vista {

constexpr double kC = 299792458.0;  // speed of light [m/s]

// One input channel of one target, after host planning.
//   a    = nu_k / c, so u_lambda = u_m * a (the rest-frame scaling of Eq. 1 cancels:
//          (u_m / (1+z)) * (nu_k (1+z) / c));
//   j0   = first rest channel of the overlap set J_k (Eq. 4), nj = |J_k| (0: outside);
//   foff = offset of the nj overlap fractions f_kj in the target's fraction array.
struct DevChan {
    double a;
    int32_t j0;
    int32_t nj;
    int32_t foff;
    int32_t pad;
};

// One target as the kernels see it.  Row g of the launch's row space is row
// g - row_base of the target whose [row_base, row_base + nrow) holds it.
struct DevTarget {
    const double* uvw;        // [nrow][3]
    const float2* vis;        // [nrow][nchan][npol]
    const float* weight;      // [nrow][npol] or [nrow][nchan][npol]
    const uint8_t* flag;      // [nrow][nchan][npol] or nullptr
    const DevChan* chan;      // [nchan]
    const float* fval;        // overlap fractions
    const int32_t* blk;       // [nblk][2]: k range [lo, hi) of the channels that reach
                              // rest-channel block b (block size = the launch's jsub)
    const int32_t* inband;    // [nchan+1] prefix count of channels with nj > 0
    int64_t row_base;
    int64_t nrow;
    int32_t nchan, npol, weight_per_chan, stack;
    int32_t kin_lo, kin_hi;   // hull of the channels with nj > 0
    int32_t nphase;           // lanes this many channels apart never share a rest channel
    int32_t pad;
    double l, m, nm1;         // direction cosines, n - 1
};

// One stack (grid) of a launch.
struct DevStack {
    int32_t nu, nv, nchan;
    int32_t tiles_u, tiles_v;
    int32_t nblocks;          // rest-channel blocks of size jc
    int32_t target_begin, target_end;
    int64_t tile_base;        // first global tile id of this stack
    double inv_du, inv_dv;
    float2* out_vis;          // [nchan][nv][nu] or nullptr
    float* out_w;
    uint32_t* out_cnt;
    double2* out_vis64;
    double* out_w64;
    unsigned long long* stats;  // [8]: samples, flagged, bad weight, outside uv,
                                //      outside band, used, contrib, overflow flag
    // carried grid state for multi-wave runs (nullptr for a single pass)
    float* st_s;              // [3][nchan][nv][nu]: re, im, w
    float* st_c;              // [3][nchan][nv][nu]: Kahan compensations
    uint32_t* st_n;           // [nchan][nv][nu]
};

struct LaunchDesc {
    const DevTarget* targets;
    const DevStack* stacks;
    const int64_t* target_row_base;   // [ntargets+1]
    const int64_t* stack_tile_base;   // [nstacks+1]
    int32_t ntargets, nstacks;
    int32_t tu, tv, jc, jsub;         // tile, block, ordered sub-block
    int64_t nrows;                    // rows in the launch
    int32_t mode;                     // kModeAtomic / kModeOrdered
    int32_t phase_fp32;
    int32_t carry;                    // 0: write outputs; 1: merge into carried state
    int32_t last_wave;                // with carry: also write outputs
    int32_t kahan;
};

constexpr int kModeAtomic = 0;
constexpr int kModeOrdered = 1;

// Kernel launchers (vista_kernels.hip).  All enqueue on `stream` and return the first
// HIP error.
// Binning pass over every row of the launch: emit == 0 counts the (row, tile) records
// of each row into seg_count and adds the outside-uv samples to the stacks' stats;
// emit == 1 writes the records at seg_off.
hipError_t launch_track(const LaunchDesc& L, const LaunchDesc* dL, uint64_t* seg_count,
                        const uint64_t* seg_off, uint32_t* keys, uint64_t* vals, int emit,
                        hipStream_t stream);
hipError_t launch_exclusive_scan_u64(const uint64_t* in, uint64_t* out, int64_t n, void* tmp,
                                     size_t* tmp_bytes, hipStream_t stream);
hipError_t launch_sort_pairs(const uint32_t* kin, uint32_t* kout, const uint64_t* vin, uint64_t* vout,
                             int64_t n, int end_bit, void* tmp, size_t* tmp_bytes, hipStream_t stream);
hipError_t launch_tile_offsets(const uint32_t* sorted_keys, int64_t nrec, int64_t ntiles,
                               uint32_t* tile_off, uint64_t* tile_cost, const uint64_t* vals,
                               hipStream_t stream);
// The accumulation over `nunits` (global tile, rest-channel block) units; the grid is
// `grid` workgroups of `waves` wavefronts that pull units from *counter (zeroed first).
hipError_t launch_accum_impl(const LaunchDesc& L, const LaunchDesc* dL, const uint2* units,
                             int64_t nunits, uint32_t* counter, const uint32_t* tile_off,
                             const uint64_t* recs, int grid, int waves, hipStream_t stream);
int accum_max_blocks_per_cu(int tu, int tv, int jc, int waves, int mode, int kahan, int npol);
size_t accum_lds_bytes(int tu, int tv, int jc, int mode, int kahan);
bool accum_shape_supported(int tu, int tv, int jc, int waves, int mode, int kahan);
hipError_t launch_debug_indices(const DevTarget* t, const DevStack* s, int32_t* iu, int32_t* iv,
                                int32_t* j0, int32_t* nj, int64_t nrow, int32_t nchan,
                                hipStream_t stream);
hipError_t launch_debug_rotate(const DevTarget* t, float2* out, int64_t nrow, int32_t nchan, int32_t npol,
                               int phase_fp32, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t stream);

}  // namespace vista
