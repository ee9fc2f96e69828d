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
//   jn   = j0 | nj << 24: j0 the first rest channel of the overlap set J_k (Eq. 4), nj =
//          |J_k| (0: outside the band; J_k is the contiguous range [j0, j0 + nj));
//   f0   = the first overlap fraction f_kj (Eq. 4).  The second is in the target's f1
//          array, all nj of them at foff[k] in its fval array (read only when nj > 2).
struct DevChan {
    double a;
    uint32_t jn;
    float f0;
};
constexpr uint32_t kJMask = 0xffffffu;
constexpr int kMaxNj = 255;

// One target as the kernels see it.  Row g of the launch's row space is row
// g - row_base of the target whose [row_base, row_base + nrow) holds it.
struct DevTarget {
    const double* uvw;        // [nrow][3]
    const float2* vis;        // [nrow][nchan][npol]
    const float* weight;      // [nrow][npol] or [nrow][nchan][npol]
    const uint8_t* flag;      // [nrow][nchan][npol] or nullptr
    const DevChan* chan;      // [nchan]
    const float* f1;          // [nchan] second overlap fraction
    const int32_t* foff;      // [nchan] offset of channel k's fractions in fval
    const float* fval;        // overlap fractions
    const int32_t* blk;       // [nblocks][2]: k range [lo, hi) of the channels that reach
                              // rest-channel block b (block size = the launch's jc)
    const int32_t* sblk;      // the same for sub-blocks of size jsub (ordered mode)
    const int32_t* inband;    // [nchan+1] prefix count of channels with nj > 0
    int64_t row_base;
    int64_t nrow;
    int32_t nchan, npol, weight_per_chan, stack;
    int32_t kin_lo, kin_hi;   // hull of the channels with nj > 0
    int32_t nphase;           // lanes this many channels apart never share a rest channel
    int32_t nblocks;          // entries of blk
    int32_t chan0;            // index of channel 0 in the launch-wide channel tables
    double l, m, nm1;         // direction cosines, n - 1
    double rot[6];            // with `rotate`: the first two rows of Eq. 1's R (uv cells from
                              // R (u, v, w)); the Eq. 2 phase keeps the original baseline
    int32_t rotate, pad_rot;
};

// Context of row g of a launch, written once by the binning pass and read by the
// accumulation kernels for every record of the row.
struct RowCtx {
    double U, V;              // uvw[r][0], uvw[r][1] [m]
    double T;                 // U l + V m + W (n - 1) [m]: channel k's Eq. 2 phase is T a_k
                              // turns (under the FP32-phase ablation: formed in FP32)
    float w0, w1;             // row weights of polarisations 0 and 1 (npol == 2, row weights)
    uint64_t vis;             // address of vis[r][0][0]
    uint64_t flag;            // address of flag[r][0][0]; a zero row when there are no flags
    uint64_t wrow;            // address of the row's first weight
    int32_t chan0;            // launch-wide index of the target's channel 0
    uint32_t info;            // npol | weight_per_chan << 8
};
static_assert(sizeof(RowCtx) == 64, "RowCtx is one 64-byte record");

// One stack (grid) of a launch.
struct DevStack {
    int32_t nu, nv, nchan;
    int32_t tiles_u, tiles_v;
    int32_t nblocks;          // rest-channel blocks of size jc
    int32_t target_begin, target_end;
    int64_t tile_base;        // first global tile id of this stack
    int64_t unit_base;        // first global (tile, block) unit id: unit_base + tile*nblocks + b
    double inv_du, inv_dv;
    float2* out_vis;          // [nchan][nv][nu] or nullptr
    float* out_w;
    uint32_t* out_cnt;
    double2* out_vis64;
    double* out_w64;
    unsigned long long* stats;  // [8]: samples, flagged, bad weight, outside uv,
                                //      outside band, used, contrib, overflow flag
    // grid state carried across the waves of a streamed batch (nullptr otherwise), laid
    // out unit by unit: unit u = tile * nblocks + b holds its tu x tv x jc cells at
    // [u][jl][lv][lu], so that a unit reads and writes its state as one contiguous block
    float* st_s;              // [3][st_plane]: re, im, w
    float* st_c;              // [3][st_plane]: Kahan compensations
    uint32_t* st_n;           // [st_plane]
    int64_t st_plane;         // tiles_u * tiles_v * nblocks * tu * tv * jc
    int32_t carry;            // 1: merge this launch's sums into the carried state
    int32_t last;             // with carry: this is the stack's last wave, write outputs
};

struct LaunchDesc {
    const DevTarget* targets;
    const DevStack* stacks;
    const int64_t* target_row_base;   // [ntargets+1]
    const int64_t* stack_tile_base;   // [nstacks+1]
    const int64_t* stack_unit_base;   // [nstacks+1]
    int32_t ntargets, nstacks;
    int32_t tu, tv, jc, jsub;         // tile, block, ordered sub-block
    int64_t nrows;                    // rows in the launch
    int32_t mode;                     // kModeAtomic / kModeOrdered
    int32_t phase_fp32;
    int32_t kahan;                    // carried-state merges are compensated
    int64_t nunits;                   // (tile, block) units of the launch's stacks
    // launch-wide channel tables (targets' tables are slices at their chan0) and row contexts
    const DevChan* chan_all;
    const float* f1_all;
    const int32_t* foff_all;          // offsets into fval_all
    const float* fval_all;
    RowCtx* rowctx;                   // [nrows]
    int32_t* row_target;              // [nrows] each row's target (ordered mode; else null)
    const uint8_t* zero_flags;        // a zero row for targets without flags
};

// One target of a rebinning launch (per-row product): its inputs, outputs and tables.
//   a[k]      = nu_k / c;
//   jstart    = [nout+1] CSR offsets, per output channel j, into ek/ef: the input channels
//               k (ascending) whose Eq. 4 fraction f_kj with channel j is above the sliver
//               threshold, and those fractions.
struct RebinTarget {
    const double* uvw;        // [nrow][3]
    const float2* vis;        // [nrow][nchan][npol]
    const uint8_t* flag;      // [nrow][nchan][npol] or nullptr
    float2* out_vis;          // [nrow][nout][npol]
    uint8_t* out_flag;        // [nrow][nout][npol] or nullptr
    float* out_wsum;          // [nrow][nout][npol] or nullptr
    double* out_uvw;          // [nrow][3] or nullptr
    const double* a;
    const int32_t* jstart;
    const int32_t* ek;
    const float* ef;
    int64_t nrow;
    int32_t nchan, npol, nout, pad;
    double l, m, nm1, opz;    // direction cosines, n - 1, 1 + z
    double R[9];              // Eq. 1's rotation (with `rotate`) of the output baselines
    int32_t rotate, pad_rot;
};
// A workgroup's share: rows [row0, row0 + nrows) of target `target`.
struct RebinBlock {
    int32_t target, row0, nrows, pad;
};

constexpr int kModeAtomic = 0;
constexpr int kModeOrdered = 1;

// Kernel launchers (vista_kernels.hip, vista_accum.hip).  All enqueue on `stream` and
// return the first HIP error.
// Binning pass over every row of the launch.  emit == 0 counts the records of each row
// into seg_count and adds the outside-uv samples to the stacks' stats; emit == 1 writes
// them at seg_off: key = global (tile, block) unit, value = row << 32 | k_lo << 16 | k_hi,
// one record per run of channels of one row inside one uv tile and one rest-channel
// block.
hipError_t launch_track(int64_t rows_cap, const LaunchDesc* dL, uint32_t* seg_count,
                        const uint32_t* seg_off, uint32_t* keys, uint64_t* vals, int emit,
                        hipStream_t stream);
// unit_off[u] = first record of unit u in the sorted keys (u = 0..nunits).  Counts are
// read from device memory (nrec_dev, nunits_dev); capacities size the grids.
hipError_t launch_unit_offsets(const uint32_t* sorted_keys, const int64_t* nrec_dev, int64_t nrec_cap,
                               const int64_t* nunits_dev, int64_t units_cap, uint32_t* unit_off,
                               hipStream_t stream);
// Per-record prefix of the records' channel counts: pre[i] = sum of (k_hi - k_lo) over the
// sorted records before i (pre[nrec] = total); lens is nrec u32 of scratch.
hipError_t launch_record_prefix(const uint64_t* recs, const int64_t* nrec_dev, int64_t nrec_cap, uint32_t* lens,
                                uint64_t* pre, uint64_t* sums, hipStream_t stream);
// Work list of the accumulation (keys/vals: nunits entries each, sorted in place;
// vals end as the unit ids).  One stack in the launch (dL->nstacks): units above four times
// the mean channel-sample count first, largest first, then the rest in unit order; several
// stacks: all units by descending channel-sample count.
hipError_t launch_unit_order(const LaunchDesc* dL, const uint32_t* unit_off, const uint64_t* pre,
                             const int64_t* nunits_dev, int64_t nunits_cap, uint32_t* keys, uint64_t* vals,
                             void* sort_temp, hipStream_t stream);
// The packed accumulation (atomic mode): `grid` workgroups of `waves` wavefronts pull units
// from *counter (zeroed first) in the order of `order` (u64 unit ids, L.nunits of them).
// acc32: per-tile sums in FP32 (the plain FP32 form) instead of FP64.  agg: runs of lanes
// adding to one cell are summed across the wavefront before they reach LDS (launches of
// mostly fine channels, where many consecutive channels share a rest channel and a cell).
hipError_t launch_accum_packed(const LaunchDesc& L, const LaunchDesc* dL, const uint64_t* order, uint32_t* counter,
                               const uint32_t* unit_off, const uint64_t* recs, const uint64_t* pre, int grid, int waves,
                               int npol, int acc32, int agg, hipStream_t stream);
int accum_packed_max_blocks_per_cu(int tu, int tv, int jc, int waves, int npol, int acc32, int agg);
bool accum_packed_shape_supported(int tu, int tv, int jc, int waves, int acc32);
int accum_packed_shape_list(int acc32, int* tu, int* tv, int* jc, int cap);
size_t accum_packed_lds_bytes(int tu, int tv, int jc, int acc32);
// The ordered accumulation (deterministic modes) over the work list `order` (global unit
// ids); `grid` workgroups of `waves` wavefronts pull list entries from *counter (zeroed
// first).  It reads the count pass's row contexts and row targets (L.rowctx,
// L.row_target).  npol == 2 when every target of the launch has two polarisations and row
// weights (specialised path).
hipError_t launch_accum_impl(const LaunchDesc& L, const LaunchDesc* dL, const uint64_t* order,
                             uint32_t* counter, const uint32_t* unit_off,
                             const uint64_t* recs, int grid, int waves, int npol, hipStream_t stream);
int accum_max_blocks_per_cu(int tu, int tv, int jc, int waves, int mode, int kahan, int npol);
size_t accum_lds_bytes(int tu, int tv, int jc, int mode, int kahan);
bool accum_shape_supported(int tu, int tv, int jc, int waves, int mode, int kahan);

// Scan and sort (vista_sort.hip).  Counts are read from device memory when n_dev is not
// null; `cap` sizes the grid.  No memset, no synchronisation: graph-capturable.
size_t scan_temp_elems(int64_t cap);
hipError_t exclusive_scan_u32_to_u32(const uint32_t* in, const int64_t* n_dev, int64_t cap, uint32_t* out,
                                     uint64_t* sums, hipStream_t s);
hipError_t exclusive_scan_u64(const uint64_t* in, const int64_t* n_dev, int64_t cap, uint64_t* out,
                              uint64_t* sums, hipStream_t s);
hipError_t exclusive_scan_u32_to_u64(const uint32_t* in, const int64_t* n_dev, int64_t cap, uint64_t* out,
                                     uint64_t* sums, hipStream_t s);
size_t radix_sort_temp_bytes(int64_t cap);
// Stable sort of (keys, vals) by the low `bits` bits of the keys, in place.
hipError_t radix_sort_pairs(uint32_t* keys, uint64_t* vals, const int64_t* n_dev, int64_t cap, int bits,
                            void* temp, hipStream_t s);
hipError_t launch_debug_indices(const DevTarget* t, const DevStack* s, int32_t* iu, int32_t* iv,
                                int32_t* j0, int32_t* nj, int64_t nrow, int32_t nchan,
                                hipStream_t stream);
hipError_t launch_copy16(void* dst, const void* src, int64_t n16, hipStream_t stream);
hipError_t launch_debug_rotate(const DevTarget* t, float2* out, int64_t nrow, int32_t nchan, int32_t npol,
                               int phase_fp32, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t stream);
// *flag |= 1 when a and b differ anywhere in [0, n) (the caller zeroes *flag).
hipError_t launch_diff_u32(const uint32_t* a, const uint32_t* b, int64_t n, uint32_t* flag, hipStream_t stream);
// Launch shapes of the accumulation of `mode`, in order: the ordered kernel's, or for the
// atomic mode the packed kernel's FP64-sum shapes.
int accum_shape_list(int mode, int* tu, int* tv, int* jc, int cap);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t stream);
// Dirty image of every channel of a stacked grid (vista_image.hip): nu, nv powers of two
// in 2..4096; tmp holds tmp_bytes (at least one nu x nv complex plane; the channels are
// imaged in passes of as many planes as it holds: image_temp_bytes(nu, nv, nchan) is one
// pass), wsum nchan doubles; beam may be null.
size_t image_temp_bytes(int nu, int nv, int nchan);
hipError_t launch_image(const void* sum_wvis, const float* sum_w, float* image, float* beam, int nu, int nv,
                        int nchan, float2* tmp, size_t tmp_bytes, double* wsum, hipStream_t stream);
// The no-alloc imaging scratch: kNoAllocImageStaging bytes of staging planes, then
// kNoAllocImageWsum bytes of weight sums (65535 doubles), 256-byte aligned.  Returns the
// current device's address of it (looked up once per device), or nullptr with *err set.
constexpr size_t kNoAllocImageStaging = (size_t)64 << 20;
constexpr size_t kNoAllocImageWsum = (size_t)512 << 10;
constexpr int kMaxDevices = 64;
void* image_noalloc_scratch(hipError_t* err);
// The per-row rebinning (vista_rebin.hip) over `nblocks` row blocks; every target of the
// launch has `npol` polarisations (1, 2 or 4).
hipError_t launch_rebin_rows(const RebinTarget* targets, const RebinBlock* blocks, int64_t nblocks, int npol,
                             hipStream_t stream);

}  // namespace vista
