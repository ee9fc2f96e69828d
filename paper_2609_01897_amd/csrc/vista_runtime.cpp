// Host runtime and C ABI of the ViSta stacking library: handles, validation, device
// residency of the inputs, and the launch sequence
//   tracks (count) -> scan -> tracks (emit) -> sort by tile -> tile offsets/costs ->
//   work list (heaviest tiles first) -> LDS accumulation (writes every output cell once).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "vista.h"
#include "vista_internal.h"
#include "vista_plan.h"

namespace vista {

// --------------------------------------------------------------------------- errors

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

struct HipFail {
    hipError_t e;
    std::string where;
};

#define VISTA_HIP(call)                                                              \
    do {                                                                             \
        hipError_t _e = (call);                                                      \
        if (_e != hipSuccess) throw HipFail{_e, std::string(#call)};                  \
    } while (0)

struct NoMem {
    std::string what;
};

// ------------------------------------------------------------- allocation and faults

// VISTA_DEVICE_MEM_LIMIT caps the bytes the library holds on the device at once, and
// VISTA_FAULT_INJECT=alloc|launch makes the next device allocation or kernel launch
// fail, so the failure paths can be exercised from the host.
struct Env {
    int64_t mem_limit = -1;
    bool fail_alloc = false;
    bool fail_launch = false;
};

static Env read_env() {
    Env e;
    if (const char* s = getenv("VISTA_DEVICE_MEM_LIMIT")) e.mem_limit = atoll(s);
    if (const char* s = getenv("VISTA_FAULT_INJECT")) {
        e.fail_alloc = strstr(s, "alloc") != nullptr;
        e.fail_launch = strstr(s, "launch") != nullptr;
    }
    return e;
}

static std::atomic<int64_t> g_dev_bytes{0};

static void pool_setup_once() {
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return;
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess) return;
        uint64_t thr = UINT64_MAX;  // keep freed blocks cached for the next launch
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    });
}

// Stream-ordered device buffers owned by one launch or handle.
class DevMem {
  public:
    explicit DevMem(hipStream_t s) : s_(s) {}
    DevMem(const DevMem&) = delete;
    ~DevMem() { release(); }
    void* alloc(size_t n) {
        if (n == 0) n = 16;
        Env e = read_env();
        if (e.fail_alloc) throw NoMem{"injected allocation failure"};
        if (e.mem_limit >= 0 && g_dev_bytes.load() + (int64_t)n > e.mem_limit)
            throw NoMem{"device memory limit reached"};
        pool_setup_once();
        void* p = nullptr;
        hipError_t r = hipMallocAsync(&p, n, s_);
        if (r == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            throw NoMem{"device allocation of " + std::to_string(n) + " bytes failed"};
        }
        if (r != hipSuccess) throw HipFail{r, "hipMallocAsync"};
        g_dev_bytes += (int64_t)n;
        ptrs_.push_back({p, n});
        return p;
    }
    template <class T>
    T* alloc_n(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
    void release() {
        for (auto& q : ptrs_) {
            (void)hipFreeAsync(q.first, s_);
            g_dev_bytes -= (int64_t)q.second;
        }
        ptrs_.clear();
    }

  private:
    hipStream_t s_;
    std::vector<std::pair<void*, size_t>> ptrs_;
};

static void check_launch(hipError_t e, const char* what) {
    if (read_env().fail_launch) throw HipFail{hipErrorLaunchFailure, std::string("injected launch failure: ") + what};
    if (e == hipErrorInvalidValue) throw HipFail{e, std::string("unsupported launch shape: ") + what};
    if (e != hipSuccess) throw HipFail{e, what};
}

// ------------------------------------------------------------------------ handles

struct HostTarget {
    vista_target t{};
    ChannelPlan plan;
    std::vector<double> freq, width;
    std::vector<unsigned char> staging;   // VISTA_MEM_HOST data: uvw | vis | weight | flag
    uint64_t n_samples = 0, n_outside_band = 0;
};

static void copy_target(HostTarget& h, const vista_grid_desc* g, const vista_target* t) {
    h.t = *t;
    h.freq.assign(t->chan_freq, t->chan_freq + t->nchan);
    h.t.chan_freq = h.freq.data();
    if (t->chan_width) {
        h.width.assign(t->chan_width, t->chan_width + t->nchan);
        h.t.chan_width = h.width.data();
    }
    h.plan = plan_target(g, &h.t);
    h.n_samples = (uint64_t)t->nrow * t->nchan * t->npol;
    h.n_outside_band = (uint64_t)t->nrow * t->npol * (uint64_t)(t->nchan - h.plan.n_inband);
    if (t->mem == VISTA_MEM_HOST && t->nrow > 0) {
        size_t nr = (size_t)t->nrow, ns = nr * t->nchan * t->npol;
        size_t b_uvw = nr * 3 * sizeof(double), b_vis = ns * 8;
        size_t b_w = (t->weight_per_chan ? ns : nr * t->npol) * sizeof(float);
        size_t b_f = t->flag ? ns : 0;
        auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
        h.staging.resize(up(b_uvw) + up(b_vis) + up(b_w) + up(b_f) + 256);
        unsigned char* base = h.staging.data();
        base += (256 - ((uintptr_t)base & 255)) & 255;
        unsigned char* p = base;
        memcpy(p, t->uvw, b_uvw); h.t.uvw = (const double*)p; p += up(b_uvw);
        memcpy(p, t->vis, b_vis); h.t.vis = p; p += up(b_vis);
        memcpy(p, t->weight, b_w); h.t.weight = (const float*)p; p += up(b_w);
        if (b_f) { memcpy(p, t->flag, b_f); h.t.flag = (const uint8_t*)p; }
    }
}

struct Tuning {
    int tu = 8, tv = 4, jc = 128, waves = 16, wg_per_cu = 0;
};

// Launch shapes the kernels are built for: the packed kernel's (plain mode) or the
// ordered kernel's (deterministic and compensated modes).
static bool shape_ok(const Tuning& t, uint32_t flags) {
    if (flags & (VISTA_F_DETERMINISTIC | VISTA_F_KAHAN))
        return accum_shape_supported(t.tu, t.tv, t.jc, t.waves, kModeOrdered, (flags & VISTA_F_KAHAN) ? 1 : 0);
    return accum_packed_shape_supported(t.tu, t.tv, t.jc, t.waves);
}

static Tuning default_tuning(uint32_t flags) {
    Tuning t;
    if (flags & (VISTA_F_DETERMINISTIC | VISTA_F_KAHAN)) {
        t.tu = 8; t.tv = 4; t.jc = 128; t.waves = 8;   // ordered: 16-channel slices per wave
    }
    return t;
}

static Tuning merge_tuning(Tuning base, const vista_tuning* u) {
    if (!u) return base;
    if (u->tile_u > 0) base.tu = u->tile_u;
    if (u->tile_v > 0) base.tv = u->tile_v;
    if (u->jblock > 0) base.jc = u->jblock;
    if (u->waves > 0) base.waves = u->waves;
    if (u->wg_per_cu > 0) base.wg_per_cu = u->wg_per_cu;
    return base;
}

}  // namespace vista

using namespace vista;

struct vista_stack {
    vista_grid_desc g{};
    hipStream_t stream = nullptr;
    int state = 0;   // 0 open, 1 finalized, 2 poisoned
    std::vector<std::unique_ptr<HostTarget>> targets;
    Tuning tune;
    bool tune_set = false;
    vista_timings tim{};
};

struct vista_batch {
    std::vector<vista_grid_desc> g;
    hipStream_t stream = nullptr;
    int state = 0;   // 0 open, 1 ran, 2 poisoned
    std::vector<std::vector<std::unique_ptr<HostTarget>>> targets;
    Tuning tune;
    bool tune_set = false;
    int64_t stream_budget = 0;
    vista_timings tim{};
    // results of vista_batch_run, kept on the device until finalize
    struct Result {
        float2* vis = nullptr;
        float* w = nullptr;
        uint32_t* cnt = nullptr;
        double2* vis64 = nullptr;
        double* w64 = nullptr;
        vista_stats st{};
        bool overflow = false;
    };
    std::vector<Result> res;
    std::unique_ptr<DevMem> keep;
};

namespace vista {

// ----------------------------------------------------------------- the launch sequence

struct StackJob {
    const vista_grid_desc* g;
    std::vector<HostTarget*> targets;
    vista_output out;          // device pointers (or NULL)
    vista_stats stats{};
    bool overflow = false;
};

struct Events {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    explicit Events() {
        for (auto& x : e) VISTA_HIP(hipEventCreate(&x));
    }
    ~Events() {
        for (auto& x : e)
            if (x) (void)hipEventDestroy(x);
    }
    float ms(int a, int b) {
        float t = 0;
        (void)hipEventElapsedTime(&t, e[a], e[b]);
        return t;
    }
};

static int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            cus = p.multiProcessorCount;
        if (!cus) cus = 256;
    }
    return cus;
}

// Stack every job in one pass: all output cells of every job are written.
static void run_jobs(std::vector<StackJob>& jobs, const Tuning& tu, uint32_t flags, hipStream_t stream,
                     vista_timings* tim) {
    DevMem mem(stream);
    Events ev;
    const int mode = (flags & (VISTA_F_DETERMINISTIC | VISTA_F_KAHAN)) ? kModeOrdered : kModeAtomic;
    const int kahan = (flags & VISTA_F_KAHAN) ? 1 : 0;
    if (!shape_ok(tu, flags))
        throw HipFail{hipErrorInvalidValue, "unsupported launch shape (tile/jblock/waves)"};
    const int jsub = mode == kModeOrdered ? tu.jc / tu.waves : tu.jc;

    // ---- host side: tables of every target, packed into one device upload
    std::vector<DevTarget> dts;
    std::vector<DevStack> dss(jobs.size());
    std::vector<int64_t> row_base, tile_base;
    std::vector<unsigned char> arena;
    auto put = [&arena](const void* p, size_t n) {
        size_t off = (arena.size() + 255) & ~(size_t)255;
        arena.resize(off + n);
        if (n) memcpy(arena.data() + off, p, n);
        return off;
    };
    struct Offs { size_t blk, sblk, inband; };
    // launch-wide channel tables: target i's entries start at its chan0
    std::vector<DevChan> chan_all;
    std::vector<float> f1_all, fval_all;
    std::vector<int32_t> foff_all;
    int64_t zero_flag_bytes = 0;
    std::vector<Offs> offs;
    int64_t rows = 0, tiles = 0, nunits = 0;
    std::vector<int64_t> unit_base;
    for (size_t s = 0; s < jobs.size(); ++s) {
        const vista_grid_desc* g = jobs[s].g;
        DevStack& S = dss[s];
        memset(&S, 0, sizeof(S));
        S.nu = g->nu; S.nv = g->nv; S.nchan = g->nchan;
        S.tiles_u = (g->nu + tu.tu - 1) / tu.tu;
        S.tiles_v = (g->nv + tu.tv - 1) / tu.tv;
        S.nblocks = (g->nchan + tu.jc - 1) / tu.jc;
        S.inv_du = 1.0 / g->du;
        S.inv_dv = 1.0 / g->dv;
        S.target_begin = (int32_t)dts.size();
        S.tile_base = tiles;
        S.unit_base = nunits;
        tile_base.push_back(tiles);
        unit_base.push_back(nunits);
        tiles += (int64_t)S.tiles_u * S.tiles_v;
        nunits += (int64_t)S.tiles_u * S.tiles_v * S.nblocks;
        for (HostTarget* h : jobs[s].targets) {
            if (h->t.nrow == 0) continue;
            DevTarget T;
            memset(&T, 0, sizeof(T));
            T.row_base = rows;
            T.nrow = h->t.nrow;
            T.nchan = h->t.nchan;
            T.npol = h->t.npol;
            T.weight_per_chan = h->t.weight_per_chan;
            T.stack = (int32_t)s;
            T.kin_lo = h->plan.kin_lo;
            T.kin_hi = h->plan.kin_hi;
            T.nphase = h->plan.nphase;
            T.nblocks = S.nblocks;
            T.l = h->t.l; T.m = h->t.m; T.nm1 = h->plan.nm1;
            T.chan0 = (int32_t)chan_all.size();
            chan_all.insert(chan_all.end(), h->plan.chan.begin(), h->plan.chan.end());
            f1_all.insert(f1_all.end(), h->plan.f1.begin(), h->plan.f1.end());
            for (int32_t f : h->plan.foff) foff_all.push_back(f + (int32_t)fval_all.size());
            fval_all.insert(fval_all.end(), h->plan.fval.begin(), h->plan.fval.end());
            if (!h->t.flag) zero_flag_bytes = std::max<int64_t>(zero_flag_bytes, (int64_t)h->t.nchan * h->t.npol);
            if (chan_all.size() >= 0x7fffffffu || fval_all.size() >= 0x7fffffffu)
                throw HipFail{hipErrorInvalidValue, "too many channels in one launch"};
            Offs o;
            std::vector<int32_t> blk = block_ranges(h->plan, g->nchan, tu.jc);
            o.blk = put(blk.data(), blk.size() * sizeof(int32_t));
            if (jsub != tu.jc) {
                std::vector<int32_t> sblk = block_ranges(h->plan, g->nchan, jsub);
                o.sblk = put(sblk.data(), sblk.size() * sizeof(int32_t));
            } else {
                o.sblk = o.blk;
            }
            o.inband = put(h->plan.inband.data(), h->plan.inband.size() * sizeof(int32_t));
            offs.push_back(o);
            row_base.push_back(rows);
            rows += h->t.nrow;
            dts.push_back(T);
        }
        S.target_end = (int32_t)dts.size();
    }
    row_base.push_back(rows);
    tile_base.push_back(tiles);
    unit_base.push_back(nunits);
    if (rows >= 0xffffffffLL) throw HipFail{hipErrorInvalidValue, "more than 2^32-1 rows in one launch"};
    if (nunits >= 0xffffffffLL) throw HipFail{hipErrorInvalidValue, "too many (tile, block) units in one launch"};

    VISTA_HIP(hipEventRecord(ev.e[0], stream));

    // ---- device residency of the inputs
    size_t ti = 0;
    for (size_t s = 0; s < jobs.size(); ++s) {
        for (HostTarget* h : jobs[s].targets) {
            if (h->t.nrow == 0) continue;
            DevTarget& T = dts[ti++];
            const vista_target& t = h->t;
            if (t.mem == VISTA_MEM_DEVICE) {
                T.uvw = t.uvw; T.vis = (const float2*)t.vis; T.weight = t.weight; T.flag = t.flag;
            } else {
                size_t nr = (size_t)t.nrow, ns = nr * t.nchan * t.npol;
                size_t b_w = (t.weight_per_chan ? ns : nr * t.npol) * sizeof(float);
                double* du = mem.alloc_n<double>(nr * 3);
                float2* dv = mem.alloc_n<float2>(ns);
                float* dw = (float*)mem.alloc(b_w);
                VISTA_HIP(hipMemcpyAsync(du, t.uvw, nr * 3 * sizeof(double), hipMemcpyHostToDevice, stream));
                VISTA_HIP(hipMemcpyAsync(dv, t.vis, ns * 8, hipMemcpyHostToDevice, stream));
                VISTA_HIP(hipMemcpyAsync(dw, t.weight, b_w, hipMemcpyHostToDevice, stream));
                T.uvw = du; T.vis = dv; T.weight = dw; T.flag = nullptr;
                if (t.flag) {
                    uint8_t* df = mem.alloc_n<uint8_t>(ns);
                    VISTA_HIP(hipMemcpyAsync(df, t.flag, ns, hipMemcpyHostToDevice, stream));
                    T.flag = df;
                }
            }
        }
    }
    const size_t o_chan = put(chan_all.data(), chan_all.size() * sizeof(DevChan));
    const size_t o_f1 = put(f1_all.data(), f1_all.size() * sizeof(float));
    const size_t o_foff = put(foff_all.data(), foff_all.size() * sizeof(int32_t));
    const size_t o_fval = put(fval_all.data(), fval_all.size() * sizeof(float));
    unsigned char* d_arena = mem.alloc_n<unsigned char>(std::max<size_t>(arena.size(), 1));
    VISTA_HIP(hipMemcpyAsync(d_arena, arena.data(), arena.size(), hipMemcpyHostToDevice, stream));
    const DevChan* d_chan = (const DevChan*)(d_arena + o_chan);
    const float* d_f1 = (const float*)(d_arena + o_f1);
    const int32_t* d_foff = (const int32_t*)(d_arena + o_foff);
    const float* d_fval = (const float*)(d_arena + o_fval);
    for (size_t i = 0; i < dts.size(); ++i) {
        dts[i].chan = d_chan + dts[i].chan0;
        dts[i].f1 = d_f1 + dts[i].chan0;
        dts[i].foff = d_foff + dts[i].chan0;
        dts[i].fval = d_fval;
        dts[i].blk = (const int32_t*)(d_arena + offs[i].blk);
        dts[i].sblk = (const int32_t*)(d_arena + offs[i].sblk);
        dts[i].inband = (const int32_t*)(d_arena + offs[i].inband);
    }
    unsigned long long* d_stats = mem.alloc_n<unsigned long long>(8 * jobs.size());
    check_launch(launch_fill_u64(d_stats, 0ull, 8 * (int64_t)jobs.size(), stream), "fill");
    for (size_t s = 0; s < jobs.size(); ++s) {
        DevStack& S = dss[s];
        S.stats = d_stats + 8 * s;
        S.out_vis = (float2*)jobs[s].out.sum_wvis;
        S.out_w = (float*)jobs[s].out.sum_w;
        S.out_cnt = (uint32_t*)jobs[s].out.count;
        S.out_vis64 = (double2*)jobs[s].out.sum_wvis64;
        S.out_w64 = (double*)jobs[s].out.sum_w64;
    }
    DevTarget* d_t = mem.alloc_n<DevTarget>(std::max<size_t>(1, dts.size()));
    DevStack* d_s = mem.alloc_n<DevStack>(dss.size());
    int64_t* d_rb = mem.alloc_n<int64_t>(row_base.size());
    int64_t* d_tb = mem.alloc_n<int64_t>(tile_base.size());
    int64_t* d_ub = mem.alloc_n<int64_t>(unit_base.size());
    if (!dts.empty())
        VISTA_HIP(hipMemcpyAsync(d_t, dts.data(), dts.size() * sizeof(DevTarget), hipMemcpyHostToDevice, stream));
    VISTA_HIP(hipMemcpyAsync(d_s, dss.data(), dss.size() * sizeof(DevStack), hipMemcpyHostToDevice, stream));
    VISTA_HIP(hipMemcpyAsync(d_rb, row_base.data(), row_base.size() * 8, hipMemcpyHostToDevice, stream));
    VISTA_HIP(hipMemcpyAsync(d_tb, tile_base.data(), tile_base.size() * 8, hipMemcpyHostToDevice, stream));
    VISTA_HIP(hipMemcpyAsync(d_ub, unit_base.data(), unit_base.size() * 8, hipMemcpyHostToDevice, stream));

    LaunchDesc L;
    memset(&L, 0, sizeof(L));
    L.targets = d_t;
    L.stacks = d_s;
    L.target_row_base = d_rb;
    L.stack_tile_base = d_tb;
    L.stack_unit_base = d_ub;
    L.ntargets = (int32_t)dts.size();
    L.nstacks = (int32_t)dss.size();
    L.tu = tu.tu; L.tv = tu.tv; L.jc = tu.jc; L.jsub = jsub;
    L.nrows = rows;
    L.mode = mode;
    L.kahan = kahan;
    L.phase_fp32 = (flags & VISTA_F_PHASE_FP32) ? 1 : 0;
    L.chan_all = d_chan;
    L.f1_all = d_f1;
    L.foff_all = d_foff;
    L.fval_all = d_fval;
    const bool packed = mode == kModeAtomic;
    if (packed && rows > 0) {
        L.rowctx = mem.alloc_n<RowCtx>(rows);
        if (zero_flag_bytes > 0) {
            int64_t words = (zero_flag_bytes + 3) / 4;
            uint32_t* z = mem.alloc_n<uint32_t>(words);
            check_launch(launch_fill_u32(z, 0u, words, stream), "fill");
            L.zero_flags = (const uint8_t*)z;
        }
    }
    LaunchDesc* d_L = mem.alloc_n<LaunchDesc>(1);
    VISTA_HIP(hipMemcpyAsync(d_L, &L, sizeof(L), hipMemcpyHostToDevice, stream));

    // ---- binning: records of (row, tile run, block), grouped by (tile, block) unit
    int64_t nrec = 0;
    uint32_t* unit_off = mem.alloc_n<uint32_t>(nunits + 1);
    uint64_t* vals = nullptr;
    if (rows > 0) {
        uint32_t* cnt = mem.alloc_n<uint32_t>(rows);
        uint32_t* off = mem.alloc_n<uint32_t>(rows + 1);
        uint64_t* sums = mem.alloc_n<uint64_t>(scan_temp_elems(rows));
        check_launch(launch_track(L, d_L, cnt, nullptr, nullptr, nullptr, 0, stream), "track count");
        check_launch(exclusive_scan_u32_to_u32(cnt, nullptr, rows, off, sums, stream), "scan");
        int64_t nb = (int64_t)scan_temp_elems(rows) - 1;
        uint64_t total = 0;
        VISTA_HIP(hipMemcpyAsync(&total, sums + nb, 8, hipMemcpyDeviceToHost, stream));
        VISTA_HIP(hipStreamSynchronize(stream));
        if (total >= 0xffffffffull) throw HipFail{hipErrorInvalidValue, "too many track records in one launch"};
        nrec = (int64_t)total;
        if (nrec > 0) {
            uint32_t* keys = mem.alloc_n<uint32_t>(nrec);
            vals = mem.alloc_n<uint64_t>(nrec);
            void* stmp = mem.alloc(radix_sort_temp_bytes(nrec));
            check_launch(launch_track(L, d_L, nullptr, off, keys, vals, 1, stream), "track emit");
            int bits = 1;
            while (bits < 32 && (int64_t(1) << bits) < nunits) ++bits;
            check_launch(radix_sort_pairs(keys, vals, nullptr, nrec, bits, stmp, stream), "sort");
            check_launch(launch_unit_offsets(keys, nullptr, nrec, nunits, unit_off, stream), "unit offsets");
        }
    }
    if (nrec == 0) check_launch(launch_fill_u32(unit_off, 0u, nunits + 1, stream), "fill");

    if (packed) {
        // ---- record starts in the units' sample streams, and the work list: every unit of
        // every stack (units without records still write their zero cells), most samples
        // first, all on the device
        uint64_t* pre = mem.alloc_n<uint64_t>(nrec + 1);
        {
            uint32_t* lens = mem.alloc_n<uint32_t>(std::max<int64_t>(1, nrec));
            uint64_t* sums = mem.alloc_n<uint64_t>(scan_temp_elems(nrec));
            check_launch(launch_record_prefix(vals, nrec, lens, pre, sums, stream), "record prefix");
        }
        uint32_t* okeys = mem.alloc_n<uint32_t>(std::max<int64_t>(1, nunits));
        uint64_t* order = mem.alloc_n<uint64_t>(std::max<int64_t>(1, nunits));
        void* otmp = mem.alloc(radix_sort_temp_bytes(std::max<int64_t>(1, nunits)));
        check_launch(launch_unit_order(unit_off, pre, nunits, okeys, order, otmp, stream), "unit order");
        uint32_t* counter = mem.alloc_n<uint32_t>(1);
        check_launch(launch_fill_u32(counter, 0u, 1, stream), "fill");
        if (!vals) vals = mem.alloc_n<uint64_t>(1);
        VISTA_HIP(hipEventRecord(ev.e[1], stream));
        int npol_all = 2;
        for (auto& T : dts)
            if (T.npol != 2 || T.weight_per_chan) npol_all = 0;   // the specialised path: 2 pols, row weights
        int per_cu = tu.wg_per_cu > 0 ? tu.wg_per_cu
                                      : accum_packed_max_blocks_per_cu(tu.tu, tu.tv, tu.jc, tu.waves, npol_all);
        if (per_cu < 1) per_cu = 1;
        int64_t grid = std::min<int64_t>((int64_t)per_cu * device_cus(), std::max<int64_t>(1, nunits));
        check_launch(launch_accum_packed(L, d_L, order, nunits, counter, unit_off, vals, pre, (int)grid, tu.waves,
                                         npol_all, stream),
                     "accumulate");
    } else {
    // ---- work list: every (tile, block) unit of every stack, heaviest first (units
    // without records still write their zero cells)
    std::vector<uint32_t> uoff(nunits + 1);
    VISTA_HIP(hipMemcpyAsync(uoff.data(), unit_off, (nunits + 1) * 4, hipMemcpyDeviceToHost, stream));
    VISTA_HIP(hipStreamSynchronize(stream));
    std::vector<uint32_t> order(nunits);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return uoff[a + 1] - uoff[a] > uoff[b + 1] - uoff[b]; });
    uint32_t* d_order = mem.alloc_n<uint32_t>(std::max<int64_t>(1, nunits));
    if (nunits > 0)
        VISTA_HIP(hipMemcpyAsync(d_order, order.data(), nunits * 4, hipMemcpyHostToDevice, stream));
    uint32_t* counter = mem.alloc_n<uint32_t>(1);
    check_launch(launch_fill_u32(counter, 0u, 1, stream), "fill");
    if (!vals) vals = mem.alloc_n<uint64_t>(1);

    VISTA_HIP(hipEventRecord(ev.e[1], stream));
    int npol_all = 2;
    for (auto& T : dts)
        if (T.npol != 2 || T.weight_per_chan) npol_all = 0;   // the specialised path: 2 pols, row weights
    int per_cu = tu.wg_per_cu > 0 ? tu.wg_per_cu
                                  : accum_max_blocks_per_cu(tu.tu, tu.tv, tu.jc, tu.waves, mode, kahan, npol_all);
    if (per_cu < 1) per_cu = 1;
    int64_t grid = std::min<int64_t>((int64_t)per_cu * device_cus(), std::max<int64_t>(1, nunits));
    check_launch(launch_accum_impl(L, d_L, d_order, nunits, counter, unit_off, vals, (int)grid, tu.waves, npol_all,
                                   stream),
                 "accumulate");
    }
    VISTA_HIP(hipEventRecord(ev.e[2], stream));

    std::vector<unsigned long long> st(8 * jobs.size());
    VISTA_HIP(hipMemcpyAsync(st.data(), d_stats, st.size() * 8, hipMemcpyDeviceToHost, stream));
    VISTA_HIP(hipEventRecord(ev.e[3], stream));
    VISTA_HIP(hipStreamSynchronize(stream));
    for (size_t s = 0; s < jobs.size(); ++s) {
        vista_stats& o = jobs[s].stats;
        memset(&o, 0, sizeof(o));
        for (HostTarget* h : jobs[s].targets) {
            o.n_samples += h->n_samples;
            o.n_outside_band += h->n_outside_band;
        }
        o.n_flagged = st[8 * s + 1];
        o.n_bad_weight = st[8 * s + 2];
        o.n_outside_uv = st[8 * s + 3];
        o.n_used = st[8 * s + 5];
        o.n_contrib = st[8 * s + 6];
        jobs[s].overflow = st[8 * s + 7] != 0;
    }
    if (tim) {
        tim->bin_ms = ev.ms(0, 1);
        tim->accum_ms = ev.ms(1, 2);
        tim->finalize_ms = ev.ms(2, 3);
        tim->total_ms = ev.ms(0, 3);
        tim->n_records = nrec;
        tim->n_units = nunits;
        tim->n_accum_launches = 1;
        tim->n_waves = 1;
    }
    mem.release();
}

// Resolve the user's outputs to device pointers; host outputs get device temporaries
// that are copied back afterwards.
struct OutputPlan {
    vista_output dev{};
    struct Copy { void* host; void* dev; size_t n; };
    std::vector<Copy> back;
};

static OutputPlan plan_outputs(const vista_grid_desc* g, const vista_output* o, DevMem& mem) {
    OutputPlan p;
    if (!o) return p;
    size_t nc = (size_t)g->nu * g->nv * g->nchan;
    p.dev.mem = VISTA_MEM_DEVICE;
    auto one = [&](void* u, size_t esz) -> void* {
        if (!u) return nullptr;
        if (o->mem == VISTA_MEM_DEVICE) return u;
        void* d = mem.alloc(nc * esz);
        p.back.push_back({u, d, nc * esz});
        return d;
    };
    p.dev.sum_wvis = one(o->sum_wvis, 8);
    p.dev.sum_w = one(o->sum_w, 4);
    p.dev.count = one(o->count, 4);
    p.dev.sum_wvis64 = one(o->sum_wvis64, 16);
    p.dev.sum_w64 = one(o->sum_w64, 8);
    return p;
}

static bool check_output(const vista_output* o, std::string* why) {
    if (!o) return true;
    if (o->mem != VISTA_MEM_HOST && o->mem != VISTA_MEM_HOST_PINNED && o->mem != VISTA_MEM_DEVICE) {
        *why = "output mem must be a VISTA_MEM_* value";
        return false;
    }
    if (((uintptr_t)o->sum_wvis % 8) || ((uintptr_t)o->sum_w % 4) || ((uintptr_t)o->count % 4) ||
        ((uintptr_t)o->sum_wvis64 % 16) || ((uintptr_t)o->sum_w64 % 8)) {
        *why = "output buffers must be aligned to their element size (16 for sum_wvis64)";
        return false;
    }
    return true;
}

template <class F>
static int guarded(int* state, F&& f) {
    try {
        return f();
    } catch (const NoMem& e) {
        if (state) *state = 2;
        return fail(VISTA_E_NOMEM, e.what);
    } catch (const HipFail& e) {
        if (state) *state = 2;
        return fail(VISTA_E_HIP, e.where + ": " + hipGetErrorString(e.e));
    } catch (const std::bad_alloc&) {
        if (state) *state = 2;
        return fail(VISTA_E_NOMEM, "host allocation failed");
    } catch (...) {
        if (state) *state = 2;
        return fail(VISTA_E_HIP, "unexpected internal error");
    }
}

}  // namespace vista

// ------------------------------------------------------------------------------ ABI

extern "C" {

const char* vista_last_error(void) { return g_err.c_str(); }

const char* vista_version(void) { return "vista-mi355x 0.1 (gfx950)"; }

int vista_stack_create(const vista_grid_desc* g, void* hip_stream, vista_stack** out) {
    std::string why;
    if (!out) return fail(VISTA_E_ARG, "out is NULL");
    if (!check_grid(g, &why)) return fail(VISTA_E_ARG, why);
    try {
        auto* s = new vista_stack();
        s->g = *g;
        s->stream = (hipStream_t)hip_stream;
        s->tune = default_tuning(g->flags);
        *out = s;
        return VISTA_OK;
    } catch (...) {
        return fail(VISTA_E_NOMEM, "host allocation failed");
    }
}

int vista_stack_add_target(vista_stack* s, const vista_target* t) {
    if (!s) return fail(VISTA_E_ARG, "stack is NULL");
    if (s->state != 0) return fail(VISTA_E_STATE, s->state == 1 ? "stack already finalized" : "stack is poisoned");
    std::string why;
    if (!check_target(&s->g, t, &why)) return fail(VISTA_E_ARG, why);
    return guarded(nullptr, [&]() -> int {
        auto h = std::make_unique<HostTarget>();
        copy_target(*h, &s->g, t);
        std::string w;
        if (!check_plan(h->plan, &w)) return fail(VISTA_E_ARG, w);
        s->targets.push_back(std::move(h));
        return VISTA_OK;
    });
}

int vista_stack_set_tuning(vista_stack* s, const vista_tuning* tu) {
    if (!s) return fail(VISTA_E_ARG, "stack is NULL");
    if (s->state != 0) return fail(VISTA_E_STATE, "stack is not open");
    Tuning t = merge_tuning(default_tuning(s->g.flags), tu);
    if (!shape_ok(t, s->g.flags))
        return fail(VISTA_E_ARG, "unsupported tuning (tile_u, tile_v, jblock, waves)");
    s->tune = t;
    s->tune_set = tu != nullptr;
    return VISTA_OK;
}

int vista_stack_finalize(vista_stack* s, const vista_output* o, vista_stats* st) {
    if (!s) return fail(VISTA_E_ARG, "stack is NULL");
    if (s->state != 0) return fail(VISTA_E_STATE, s->state == 1 ? "stack already finalized" : "stack is poisoned");
    std::string why;
    if (!check_output(o, &why)) return fail(VISTA_E_ARG, why);
    return guarded(&s->state, [&]() -> int {
        DevMem mem(s->stream);
        OutputPlan op = plan_outputs(&s->g, o, mem);
        std::vector<StackJob> jobs(1);
        jobs[0].g = &s->g;
        for (auto& h : s->targets) jobs[0].targets.push_back(h.get());
        jobs[0].out = op.dev;
        run_jobs(jobs, s->tune, s->g.flags, s->stream, &s->tim);
        for (auto& c : op.back)
            VISTA_HIP(hipMemcpyAsync(c.host, c.dev, c.n, hipMemcpyDeviceToHost, s->stream));
        VISTA_HIP(hipStreamSynchronize(s->stream));
        mem.release();
        VISTA_HIP(hipStreamSynchronize(s->stream));
        if (st) *st = jobs[0].stats;
        s->state = 1;
        if (jobs[0].overflow) return fail(VISTA_E_RANGE, "a cell count exceeds 2^32-1");
        return VISTA_OK;
    });
}

int vista_stack_timings(const vista_stack* s, vista_timings* t) {
    if (!s || !t) return fail(VISTA_E_ARG, "NULL argument");
    *t = s->tim;
    return VISTA_OK;
}

int vista_stack_destroy(vista_stack* s) {
    if (!s) return fail(VISTA_E_ARG, "stack is NULL");
    delete s;
    return VISTA_OK;
}

int vista_plan_spectral_grid(int32_t n_targets, const double* const* chan_freq, const double* const* chan_width,
                             const int32_t* nchan, const double* z, double central_freq, int32_t nchan_out,
                             double* freq_lo, double* dfreq) {
    if (n_targets < 1 || !chan_freq || !nchan || !z || !freq_lo || !dfreq || nchan_out < 1)
        return fail(VISTA_E_ARG, "invalid arguments");
    if (!std::isfinite(central_freq)) return fail(VISTA_E_ARG, "central_freq must be finite");
    double wmax = 0.0;
    for (int32_t i = 0; i < n_targets; ++i) {
        const double* w = chan_width ? chan_width[i] : nullptr;
        if (!chan_freq[i] || nchan[i] < 1 || (nchan[i] == 1 && !w)) return fail(VISTA_E_ARG, "invalid target channels");
        if (!(z[i] > -1.0 && std::isfinite(z[i]))) return fail(VISTA_E_ARG, "z must be finite and > -1");
        for (int32_t k = 0; k < nchan[i]; ++k) {
            double Wr = channel_width(chan_freq[i], w, nchan[i], k) * (1.0 + z[i]);
            if (!(Wr > 0 && std::isfinite(Wr))) return fail(VISTA_E_ARG, "channel widths must be finite and > 0");
            wmax = std::max(wmax, Wr);
        }
    }
    *dfreq = wmax;
    *freq_lo = central_freq - 0.5 * (double)nchan_out * wmax;
    return VISTA_OK;
}

int vista_debug_indices(const vista_grid_desc* g, const vista_target* t, void* hip_stream, int32_t* iu, int32_t* iv,
                        int32_t* j0, int32_t* nj) {
    std::string why;
    if (!check_grid(g, &why) || !check_target(g, t, &why)) return fail(VISTA_E_ARG, why);
    if (!iu || !iv || !j0 || !nj) return fail(VISTA_E_ARG, "output is NULL");
    hipStream_t stream = (hipStream_t)hip_stream;
    return guarded(nullptr, [&]() -> int {
        HostTarget h;
        copy_target(h, g, t);
        DevMem mem(stream);
        size_t n = (size_t)t->nrow * t->nchan;
        const double* duvw = t->uvw;
        if (t->mem != VISTA_MEM_DEVICE && t->nrow > 0) {
            double* d = mem.alloc_n<double>((size_t)t->nrow * 3);
            VISTA_HIP(hipMemcpyAsync(d, h.t.uvw, (size_t)t->nrow * 24, hipMemcpyHostToDevice, stream));
            duvw = d;
        }
        DevChan* dch = mem.alloc_n<DevChan>(t->nchan);
        VISTA_HIP(hipMemcpyAsync(dch, h.plan.chan.data(), t->nchan * sizeof(DevChan), hipMemcpyHostToDevice, stream));
        DevTarget T;
        memset(&T, 0, sizeof(T));
        T.uvw = duvw; T.chan = dch; T.nrow = t->nrow; T.nchan = t->nchan; T.npol = t->npol;
        DevStack S;
        memset(&S, 0, sizeof(S));
        S.nu = g->nu; S.nv = g->nv; S.nchan = g->nchan; S.inv_du = 1.0 / g->du; S.inv_dv = 1.0 / g->dv;
        DevTarget* dT = mem.alloc_n<DevTarget>(1);
        DevStack* dS = mem.alloc_n<DevStack>(1);
        VISTA_HIP(hipMemcpyAsync(dT, &T, sizeof(T), hipMemcpyHostToDevice, stream));
        VISTA_HIP(hipMemcpyAsync(dS, &S, sizeof(S), hipMemcpyHostToDevice, stream));
        int32_t* d4 = mem.alloc_n<int32_t>(4 * std::max<size_t>(n, 1));
        check_launch(launch_debug_indices(dT, dS, d4, d4 + n, d4 + 2 * n, d4 + 3 * n, t->nrow, t->nchan, stream),
                     "debug indices");
        VISTA_HIP(hipMemcpyAsync(iu, d4, n * 4, hipMemcpyDeviceToHost, stream));
        VISTA_HIP(hipMemcpyAsync(iv, d4 + n, n * 4, hipMemcpyDeviceToHost, stream));
        VISTA_HIP(hipMemcpyAsync(j0, d4 + 2 * n, n * 4, hipMemcpyDeviceToHost, stream));
        VISTA_HIP(hipMemcpyAsync(nj, d4 + 3 * n, n * 4, hipMemcpyDeviceToHost, stream));
        VISTA_HIP(hipStreamSynchronize(stream));
        mem.release();
        VISTA_HIP(hipStreamSynchronize(stream));
        return VISTA_OK;
    });
}

int vista_debug_rotate(const vista_grid_desc* g, const vista_target* t, void* hip_stream, void* out) {
    std::string why;
    if (!check_grid(g, &why) || !check_target(g, t, &why)) return fail(VISTA_E_ARG, why);
    if (!out) return fail(VISTA_E_ARG, "output is NULL");
    if (t->mem != VISTA_MEM_DEVICE) return fail(VISTA_E_ARG, "vista_debug_rotate needs device data");
    hipStream_t stream = (hipStream_t)hip_stream;
    return guarded(nullptr, [&]() -> int {
        HostTarget h;
        copy_target(h, g, t);
        DevMem mem(stream);
        DevChan* dch = mem.alloc_n<DevChan>(t->nchan);
        VISTA_HIP(hipMemcpyAsync(dch, h.plan.chan.data(), t->nchan * sizeof(DevChan), hipMemcpyHostToDevice, stream));
        DevTarget T;
        memset(&T, 0, sizeof(T));
        T.uvw = t->uvw; T.vis = (const float2*)t->vis; T.chan = dch; T.nrow = t->nrow; T.nchan = t->nchan;
        T.npol = t->npol; T.l = t->l; T.m = t->m; T.nm1 = h.plan.nm1;
        DevTarget* dT = mem.alloc_n<DevTarget>(1);
        VISTA_HIP(hipMemcpyAsync(dT, &T, sizeof(T), hipMemcpyHostToDevice, stream));
        check_launch(launch_debug_rotate(dT, (float2*)out, t->nrow, t->nchan, t->npol,
                                         (g->flags & VISTA_F_PHASE_FP32) ? 1 : 0, stream),
                     "debug rotate");
        VISTA_HIP(hipStreamSynchronize(stream));
        mem.release();
        VISTA_HIP(hipStreamSynchronize(stream));
        return VISTA_OK;
    });
}

int vista_debug_copy(void* dst, const void* src, size_t nbytes, void* hip_stream) {
    if (!dst || !src) return fail(VISTA_E_ARG, "NULL pointer");
    if ((nbytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
        return fail(VISTA_E_ARG, "vista_debug_copy needs 16-byte aligned pointers and size");
    const uintptr_t d = (uintptr_t)dst, s = (uintptr_t)src;
    if (d < s + nbytes && s < d + nbytes) return fail(VISTA_E_ARG, "regions overlap");
    return guarded(nullptr, [&]() -> int {
        check_launch(launch_copy16(dst, src, (int64_t)(nbytes / 16), (hipStream_t)hip_stream), "copy");
        return VISTA_OK;
    });
}

// ---------------------------------------------------------------------------- batch

int vista_batch_create(int32_t n_stacks, const vista_grid_desc* g, void* hip_stream, vista_batch** out) {
    if (!out) return fail(VISTA_E_ARG, "out is NULL");
    if (n_stacks < 1 || !g) return fail(VISTA_E_ARG, "need n_stacks >= 1 grids");
    std::string why;
    const uint32_t mode_bits = VISTA_F_KAHAN | VISTA_F_DETERMINISTIC | VISTA_F_PHASE_FP32;
    for (int32_t i = 0; i < n_stacks; ++i) {
        if (!check_grid(&g[i], &why)) return fail(VISTA_E_ARG, "stack " + std::to_string(i) + ": " + why);
        if ((g[i].flags & mode_bits) != (g[0].flags & mode_bits))
            return fail(VISTA_E_ARG, "all stacks of a batch need the same KAHAN/DETERMINISTIC/PHASE_FP32 flags");
    }
    try {
        auto* b = new vista_batch();
        b->g.assign(g, g + n_stacks);
        b->stream = (hipStream_t)hip_stream;
        b->targets.resize(n_stacks);
        b->tune = default_tuning(g[0].flags);
        *out = b;
        return VISTA_OK;
    } catch (...) {
        return fail(VISTA_E_NOMEM, "host allocation failed");
    }
}

int vista_batch_add_target(vista_batch* b, int32_t stack, const vista_target* t) {
    if (!b) return fail(VISTA_E_ARG, "batch is NULL");
    if (b->state != 0) return fail(VISTA_E_STATE, b->state == 1 ? "batch already ran" : "batch is poisoned");
    if (stack < 0 || stack >= (int32_t)b->g.size()) return fail(VISTA_E_ARG, "stack index out of range");
    std::string why;
    if (!check_target(&b->g[stack], t, &why)) return fail(VISTA_E_ARG, why);
    return guarded(nullptr, [&]() -> int {
        auto h = std::make_unique<HostTarget>();
        copy_target(*h, &b->g[stack], t);
        std::string w;
        if (!check_plan(h->plan, &w)) return fail(VISTA_E_ARG, w);
        b->targets[stack].push_back(std::move(h));
        return VISTA_OK;
    });
}

int vista_batch_set_tuning(vista_batch* b, const vista_tuning* tu) {
    if (!b) return fail(VISTA_E_ARG, "batch is NULL");
    if (b->state != 0) return fail(VISTA_E_STATE, "batch already ran");
    Tuning t = merge_tuning(default_tuning(b->g[0].flags), tu);
    if (!shape_ok(t, b->g[0].flags))
        return fail(VISTA_E_ARG, "unsupported tuning (tile_u, tile_v, jblock, waves)");
    b->tune = t;
    b->tune_set = tu != nullptr;
    return VISTA_OK;
}

int vista_batch_set_stream_budget(vista_batch* b, int64_t bytes) {
    if (!b) return fail(VISTA_E_ARG, "batch is NULL");
    if (bytes < 0) return fail(VISTA_E_ARG, "budget must be >= 0");
    b->stream_budget = bytes;
    return VISTA_OK;
}

int vista_batch_run(vista_batch* b) {
    if (!b) return fail(VISTA_E_ARG, "batch is NULL");
    if (b->state != 0) return fail(VISTA_E_STATE, b->state == 1 ? "batch already ran" : "batch is poisoned");
    return guarded(&b->state, [&]() -> int {
        b->keep = std::make_unique<DevMem>(b->stream);
        size_t ns = b->g.size();
        b->res.assign(ns, {});
        std::vector<StackJob> jobs(ns);
        for (size_t s = 0; s < ns; ++s) {
            const vista_grid_desc& g = b->g[s];
            size_t nc = (size_t)g.nu * g.nv * g.nchan;
            auto& R = b->res[s];
            R.vis = b->keep->alloc_n<float2>(nc);
            R.w = b->keep->alloc_n<float>(nc);
            R.cnt = b->keep->alloc_n<uint32_t>(nc);
            R.vis64 = b->keep->alloc_n<double2>(nc);
            R.w64 = b->keep->alloc_n<double>(nc);
            jobs[s].g = &b->g[s];
            for (auto& h : b->targets[s]) jobs[s].targets.push_back(h.get());
            jobs[s].out.sum_wvis = R.vis;
            jobs[s].out.sum_w = R.w;
            jobs[s].out.count = R.cnt;
            jobs[s].out.sum_wvis64 = R.vis64;
            jobs[s].out.sum_w64 = R.w64;
            jobs[s].out.mem = VISTA_MEM_DEVICE;
        }
        run_jobs(jobs, b->tune, b->g[0].flags, b->stream, &b->tim);
        for (size_t s = 0; s < ns; ++s) {
            b->res[s].st = jobs[s].stats;
            b->res[s].overflow = jobs[s].overflow;
        }
        b->state = 1;
        return VISTA_OK;
    });
}

int vista_batch_finalize(vista_batch* b, int32_t stack, const vista_output* o, vista_stats* st) {
    if (!b) return fail(VISTA_E_ARG, "batch is NULL");
    if (b->state != 1) return fail(VISTA_E_STATE, b->state == 0 ? "batch has not run" : "batch is poisoned");
    if (stack < 0 || stack >= (int32_t)b->g.size()) return fail(VISTA_E_ARG, "stack index out of range");
    std::string why;
    if (!check_output(o, &why)) return fail(VISTA_E_ARG, why);
    return guarded(&b->state, [&]() -> int {
        const vista_grid_desc& g = b->g[stack];
        size_t nc = (size_t)g.nu * g.nv * g.nchan;
        auto& R = b->res[stack];
        hipMemcpyKind kind = (o && o->mem == VISTA_MEM_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (o) {
            if (o->sum_wvis) VISTA_HIP(hipMemcpyAsync(o->sum_wvis, R.vis, nc * 8, kind, b->stream));
            if (o->sum_w) VISTA_HIP(hipMemcpyAsync(o->sum_w, R.w, nc * 4, kind, b->stream));
            if (o->count) VISTA_HIP(hipMemcpyAsync(o->count, R.cnt, nc * 4, kind, b->stream));
            if (o->sum_wvis64) VISTA_HIP(hipMemcpyAsync(o->sum_wvis64, R.vis64, nc * 16, kind, b->stream));
            if (o->sum_w64) VISTA_HIP(hipMemcpyAsync(o->sum_w64, R.w64, nc * 8, kind, b->stream));
        }
        VISTA_HIP(hipStreamSynchronize(b->stream));
        if (st) *st = R.st;
        if (R.overflow) return fail(VISTA_E_RANGE, "a cell count exceeds 2^32-1");
        return VISTA_OK;
    });
}

int vista_batch_timings(const vista_batch* b, vista_timings* t) {
    if (!b || !t) return fail(VISTA_E_ARG, "NULL argument");
    *t = b->tim;
    return VISTA_OK;
}

int vista_batch_destroy(vista_batch* b) {
    if (!b) return fail(VISTA_E_ARG, "batch is NULL");
    if (b->keep) {
        b->keep->release();
        (void)hipStreamSynchronize(b->stream);
    }
    delete b;
    return VISTA_OK;
}

int vista_stack_autotune(vista_stack* s, vista_tuning* best) {
    if (!s) return fail(VISTA_E_ARG, "stack is NULL");
    return fail(VISTA_E_STATE, "autotuning is not available in this build");
}

}  // extern "C"
