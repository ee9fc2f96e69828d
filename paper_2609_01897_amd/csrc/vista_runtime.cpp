// Host runtime and C ABI of the ViSta stacking library: handles, validation, device
// residency of the inputs, and the launch sequence
//   tracks (count) -> scan -> tracks (emit) -> sort by tile -> tile offsets/costs ->
//   work list (heaviest tiles first) -> LDS accumulation (writes every output cell once).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <condition_variable>
#include <deque>
#include <exception>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include <unistd.h>

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

// A launch's fault bits (its stacks' statistics slot 7): 1 = some cell took 2^32 or more
// contributions, so its count may have wrapped; 2 = the ordered accumulation gave up on
// ordering a chunk's additions (it bounds its turns; this cannot happen while each turn
// lets the highest bidder add).
static int fault_fail(uint64_t bits) {
    if (bits & 1u) return fail(VISTA_E_RANGE, "a cell count exceeds 2^32-1");
    return fail(VISTA_E_HIP, "the ordered accumulation left a chunk's additions unordered");
}

struct HipFail {
    hipError_t e;
    std::string where;
};

// Upper bound (exclusive) on the rows, units and track records of one launch.
constexpr int64_t kMaxItems = 0xffffff00LL;

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

// ------------------------------------------------------------------------- logging

// VISTA_LOG=0..3 sets how much the library writes to stderr: 0 nothing (the default);
// 1 one line per stack launch and batch run (records, units, device times); 2 also the
// autotuner's candidates, the batch's wave plan and every device allocation of 1 GiB or
// more; 3 also each launch's host build.
static int log_level() {
    const char* s = getenv("VISTA_LOG");
    return s ? atoi(s) : 0;
}

static void vlog(int level, const char* fmt, ...) {
    if (log_level() < level) return;
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    fprintf(stderr, "[vista] %s\n", buf);
    fflush(stderr);
}

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

// Device blocks of 1 GiB or more that batches have released, kept for the next batch on the
// same device: memory handed back to the driver is cleared again when it is next allocated
// (about 30 GB/s here), which for a streamed batch's staging buffers and carried state costs
// seconds per batch.  A block serves a request of 4/5 of its size or more.  The blocks stay
// counted as the library's device memory until vista_release_workspace or an allocation
// that would otherwise fail frees them.
class BigBlocks {
  public:
    static constexpr size_t kMin = (size_t)1 << 30;
    static BigBlocks& get() {
        static BigBlocks b;
        return b;
    }
    void* take(size_t n, int dev, size_t* got) {
        std::lock_guard<std::mutex> lk(m_);
        size_t best = blocks_.size();
        for (size_t i = 0; i < blocks_.size(); ++i) {
            const Block& b = blocks_[i];
            if (b.dev == dev && b.n >= n && b.n - n <= b.n / 5 && (best == blocks_.size() || b.n < blocks_[best].n))
                best = i;
        }
        if (best == blocks_.size()) return nullptr;
        void* p = blocks_[best].p;
        *got = blocks_[best].n;
        blocks_.erase(blocks_.begin() + (std::ptrdiff_t)best);
        return p;
    }
    void give(void* p, size_t n, int dev) {
        std::lock_guard<std::mutex> lk(m_);
        blocks_.push_back({p, n, dev});
    }
    // Free the current device's cached blocks (waiting for the device); returns their bytes.
    int64_t release(int dev) {
        std::lock_guard<std::mutex> lk(m_);
        int64_t freed = 0;
        for (size_t i = 0; i < blocks_.size();) {
            if (blocks_[i].dev == dev) {
                (void)hipFree(blocks_[i].p);
                freed += (int64_t)blocks_[i].n;
                blocks_.erase(blocks_.begin() + (std::ptrdiff_t)i);
            } else {
                ++i;
            }
        }
        return freed;
    }

  private:
    struct Block {
        void* p;
        size_t n;
        int dev;
    };
    std::mutex m_;
    std::vector<Block> blocks_;
};

static int current_device() {
    int dev = 0;
    return hipGetDevice(&dev) == hipSuccess ? dev : 0;
}

// Stream-ordered device buffers owned by one launch or handle.
// Persistent buffers (a thread's cached launch workspace, which outlives any one stream)
// are plain device allocations instead: every call that uses them synchronises its stream
// before returning, so they are idle between calls, and freeing them waits for the device.
// With `reuse_big`, blocks of 1 GiB or more come from and go back to BigBlocks (their
// release waits for the stream first).
class DevMem {
  public:
    explicit DevMem(hipStream_t s, bool persistent = false, bool reuse_big = false)
        : s_(s), persistent_(persistent), reuse_big_(reuse_big) {}
    DevMem(const DevMem&) = delete;
    ~DevMem() { release(); }
    void set_stream(hipStream_t s) { s_ = s; }
    void* alloc(size_t n) {
        if (n == 0) n = 16;
        Env e = read_env();
        if (e.fail_alloc) throw NoMem{"injected allocation failure"};
        if (reuse_big_ && n >= BigBlocks::kMin) {
            size_t got = 0;
            const int dev = current_device();
            if (void* q = BigBlocks::get().take(n, dev, &got)) {
                big_.push_back({q, got, dev});
                return q;
            }
        }
        if (e.mem_limit >= 0 && g_dev_bytes.load() + (int64_t)n > e.mem_limit) {
            g_dev_bytes -= BigBlocks::get().release(current_device());   // cached blocks first
            if (g_dev_bytes.load() + (int64_t)n > e.mem_limit) throw NoMem{"device memory limit reached"};
        }
        void* p = nullptr;
        hipError_t r;
        const bool big = n >= ((size_t)1 << 30) && log_level() >= 2;
        const auto t0 = std::chrono::steady_clock::now();
        size_t fr = 0, tot = 0;
        if (big) (void)hipMemGetInfo(&fr, &tot);
        const bool big_block = reuse_big_ && n >= BigBlocks::kMin;
        if (persistent_ || big_block) {
            r = hipMalloc(&p, n);
            if (r == hipErrorOutOfMemory && big_block) {          // the cached blocks make room
                (void)hipGetLastError();
                g_dev_bytes -= BigBlocks::get().release(current_device());
                r = hipMalloc(&p, n);
            }
        } else {
            pool_setup_once();
            r = hipMallocAsync(&p, n, s_);
        }
        if (big)
            vlog(2, "device allocation of %.2f GiB (%.2f GiB free before): %.1f ms", n / 1073741824.0,
                 fr / 1073741824.0,
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        if (r == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            throw NoMem{"device allocation of " + std::to_string(n) + " bytes failed"};
        }
        if (r != hipSuccess) throw HipFail{r, persistent_ ? "hipMalloc" : "hipMallocAsync"};
        g_dev_bytes += (int64_t)n;
        if (big_block) big_.push_back({p, n, current_device()});
        else ptrs_.push_back({p, n});
        return p;
    }
    template <class T>
    T* alloc_n(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
    void release() {
        for (auto& q : ptrs_) {
            if (persistent_) (void)hipFree(q.first);
            else (void)hipFreeAsync(q.first, s_);
            g_dev_bytes -= (int64_t)q.second;
        }
        ptrs_.clear();
        if (!big_.empty()) {
            (void)hipStreamSynchronize(s_);                // the stream's last use has passed
            for (auto& q : big_) BigBlocks::get().give(q.p, q.n, q.dev);
            big_.clear();
        }
    }

  private:
    hipStream_t s_;
    bool persistent_, reuse_big_;
    struct Big {
        void* p;
        size_t n;
        int dev;                                     // the device it was allocated on
    };
    std::vector<std::pair<void*, size_t>> ptrs_;
    std::vector<Big> big_;
};

// Enqueue a kernel launch and check it.  An injected launch failure is raised before the
// kernel is enqueued, so nothing is left running on memory the unwinding frees.
template <class F>
static void check_launch_f(F&& launch, const char* what) {
    if (read_env().fail_launch) throw HipFail{hipErrorLaunchFailure, std::string("injected launch failure: ") + what};
    const hipError_t e = launch();
    if (e == hipErrorInvalidValue) throw HipFail{e, std::string("unsupported launch shape: ") + what};
    if (e != hipSuccess) throw HipFail{e, what};
}
#define check_launch(expr, what) check_launch_f([&]() { return (expr); }, what)

// ------------------------------------------------------------------------ handles

struct HostTarget {
    vista_target t{};
    const vista_grid_desc* g = nullptr;   // the grid it is planned on (owned by its handle)
    bool planned = false;
    ChannelPlan plan;
    std::vector<double> freq, width;
    std::vector<unsigned char> staging;   // VISTA_MEM_HOST data: uvw | vis | weight | flag
    uint64_t n_samples = 0, n_outside_band = 0;
    // planning handed to the planning pool when the target was added
    std::mutex pm;
    std::condition_variable pcv;
    int pstate = 0;                       // 0 not handed over, 1 queued or running, 2 done
    std::exception_ptr perr;
    ~HostTarget() {
        std::unique_lock<std::mutex> lk(pm);
        pcv.wait(lk, [this] { return pstate != 1; });
    }
};

static void finish_plan(HostTarget& h) {
    h.plan = plan_target(h.g, &h.t);
    h.n_outside_band = (uint64_t)h.t.nrow * h.t.npol * (uint64_t)(h.t.nchan - h.plan.n_inband);
    h.planned = true;
}

// Host threads that plan the targets handed over by add_target, so that planning runs while
// the caller goes on adding targets.  Created on first use and never destroyed (its threads
// wait for work until the process ends); a forked child, which has none of them, builds its
// own.
class PlanPool {
public:
    // The pool, or nullptr when no thread could be started (callers then plan at launch).
    static PlanPool* get() {
        static std::mutex m;
        static PlanPool* pool = nullptr;
        std::lock_guard<std::mutex> lk(m);
        if (!pool || pool->pid_ != getpid()) {
            PlanPool* p = new PlanPool();
            if (!p->start()) return nullptr;            // nothing waits on it: left alone
            pool = p;
        }
        return pool;
    }
    void submit(HostTarget* h) {
        {
            std::lock_guard<std::mutex> lk(h->pm);
            h->pstate = 1;
        }
        {
            std::lock_guard<std::mutex> lk(m_);
            q_.push_back(h);
        }
        cv_.notify_one();
    }

private:
    PlanPool() : pid_(getpid()) {}
    bool start() {
        // half the cores, at most 8: planning keeps up with the caller's adds, and the
        // caller keeps a core of its own
        const unsigned n = std::min(8u, std::max(1u, std::thread::hardware_concurrency() / 2));
        unsigned started = 0;
        try {
            for (; started < n; ++started) std::thread([this] { loop(); }).detach();
        } catch (...) {
        }
        return started > 0;
    }
    void loop() {
        for (;;) {
            HostTarget* h;
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [this] { return !q_.empty(); });
                h = q_.front();
                q_.pop_front();
            }
            std::exception_ptr e;
            try {
                finish_plan(*h);
            } catch (...) {
                e = std::current_exception();
            }
            // notified under the lock: the waiter may destroy *h as soon as it is released
            std::lock_guard<std::mutex> lk(h->pm);
            h->perr = e;
            h->pstate = 2;
            h->pcv.notify_all();
        }
    }
    pid_t pid_;
    std::mutex m_;
    std::condition_variable cv_;
    std::deque<HostTarget*> q_;
};

// Hand an added target's planning to the pool (planned at launch when there is none).
static void plan_in_background(HostTarget* h) {
    if (h->planned) return;
    if (PlanPool* p = PlanPool::get()) p->submit(h);
}

// Wait for a target handed to the pool; a planning error is rethrown here, once.
static void wait_plan(HostTarget& h) {
    std::unique_lock<std::mutex> lk(h.pm);
    h.pcv.wait(lk, [&h] { return h.pstate != 1; });
    if (h.perr) {
        std::exception_ptr e = h.perr;
        h.perr = nullptr;
        h.pstate = 0;
        std::rethrow_exception(e);
    }
}

// Plan every target not yet planned, on up to 16 host threads (the channel tables of many
// targets are independent).
static void plan_all(const std::vector<HostTarget*>& hs) {
    for (HostTarget* h : hs) wait_plan(*h);        // those handed to the pool at add time
    std::vector<HostTarget*> todo;
    for (HostTarget* h : hs)
        if (!h->planned) todo.push_back(h);
    if (todo.empty()) return;
    const size_t nth = std::min<size_t>({todo.size() / 4 + 1, 16, std::max(1u, std::thread::hardware_concurrency())});
    std::atomic<size_t> next{0};
    std::vector<std::exception_ptr> err(nth);
    auto work = [&](size_t w) {
        try {
            for (size_t i; (i = next.fetch_add(1)) < todo.size();) finish_plan(*todo[i]);
        } catch (...) {
            err[w] = std::current_exception();
        }
    };
    std::vector<std::thread> pool;
    for (size_t w = 1; w < nth; ++w) pool.emplace_back(work, w);
    work(0);
    for (auto& th : pool) th.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
}

// Copy the target's description (and, for host memory, its data).  Planning waits for the
// launch, where all targets are planned together, unless the target could exceed the
// packed channel table's overlap-set limit: that is known at once, from its widest
// rest-frame channel, and such a target is planned (and checked) now.
static void copy_target(HostTarget& h, const vista_grid_desc* g, const vista_target* t, bool plan_now = false) {
    h.t = *t;
    h.g = g;
    h.freq.assign(t->chan_freq, t->chan_freq + t->nchan);
    h.t.chan_freq = h.freq.data();
    if (t->chan_width) {
        h.width.assign(t->chan_width, t->chan_width + t->nchan);
        h.t.chan_width = h.width.data();
    }
    if (!plan_now && !(g->flags & VISTA_F_SPECTRAL_NEAREST)) {
        double wmax = 0.0;
        for (int32_t k = 0; k < t->nchan; ++k)
            wmax = std::max(wmax, channel_width(h.t.chan_freq, h.t.chan_width, t->nchan, k) * (1.0 + t->z));
        plan_now = !(std::floor(wmax / g->dfreq) + 2.0 <= (double)kMaxNj);
    }
    if (plan_now) finish_plan(h);
    h.n_samples = (uint64_t)t->nrow * t->nchan * t->npol;
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
    if (flags & VISTA_F_DETERMINISTIC)
        return accum_shape_supported(t.tu, t.tv, t.jc, t.waves, kModeOrdered, (flags & VISTA_F_KAHAN) ? 1 : 0);
    return accum_packed_shape_supported(t.tu, t.tv, t.jc, t.waves, (flags & VISTA_F_PLAIN_FP32) ? 1 : 0);
}

static Tuning default_tuning(uint32_t flags) {
    Tuning t;
    if (flags & VISTA_F_DETERMINISTIC) {
        t.tu = 2; t.tv = 2; t.jc = 64; t.waves = 1;    // ordered: 16 one-wavefront workgroups a CU
    } else if (flags & VISTA_F_PLAIN_FP32) {
        t.tu = 8; t.tv = 4; t.jc = 288; t.waves = 16;  // FP32 tiles: 1.75 times the cells
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
        uint64_t overflow = 0;     // fault bits of the stack's launch (fault_fail)
    };
    std::vector<Result> res;
    std::vector<vista_output> reg;    // outputs registered before the run (mem < 0: none)
    std::unique_ptr<DevMem> keep;
};

namespace vista {

// ----------------------------------------------------------------- the launch sequence

struct StackJob {
    const vista_grid_desc* g;
    std::vector<HostTarget*> targets;
    vista_output out;          // device pointers (or NULL)
    vista_stats stats{};
    uint64_t overflow = 0;     // fault bits of the stack's launch (fault_fail)
    int32_t index = 0;         // slot of the stack's statistics
    // carried state of a stack streamed over several waves, and this launch's role
    float* st_s = nullptr;
    float* st_c = nullptr;
    uint32_t* st_n = nullptr;
    int carry = 0, last = 1;
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

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Host side of one launch: the descriptors and tables of its stacks and targets, packed
// for one upload.  Target data pointers (uvw, vis, weight, flag) are set by the caller.
// Host buffers of the launch tables, kept per thread between launches: tables of many
// targets run to tens of MB, and fresh allocations of that size come from the system
// zero-filled and fault in page by page on every launch.
struct HostScratch {
    std::vector<unsigned char> arena;         // spare arena, handed to the next launch
};
static thread_local HostScratch t_host;

struct HostLaunch {
    HostLaunch() = default;
    HostLaunch(HostLaunch&&) = default;
    HostLaunch& operator=(HostLaunch&&) = default;
    HostLaunch(const HostLaunch&) = delete;
    HostLaunch& operator=(const HostLaunch&) = delete;
    ~HostLaunch() {
        if (arena.capacity() > t_host.arena.capacity()) t_host.arena.swap(arena);
    }
    std::vector<DevTarget> dts;
    std::vector<DevStack> dss;
    std::vector<int64_t> row_base, tile_base, unit_base;
    std::vector<unsigned char> arena;
    struct Offs { size_t blk, sblk, inband; };
    std::vector<Offs> offs;
    std::vector<const HostTarget*> hts;        // the HostTarget of each DevTarget
    std::vector<int32_t> stats_index;          // per stack
    size_t o_chan = 0, o_f1 = 0, o_foff = 0, o_fval = 0;
    int64_t rows = 0, nunits = 0, zero_flag_bytes = 0;
    int npol_all = 2;
    int agg = 0;                               // wave-aggregated LDS updates (fine channels)
};

// Whether a launch takes the packed kernel's wave-aggregated LDS updates: when at least
// 30 % of its samples belong to targets whose in-band channels fall 6 or more to a rest
// channel (lanes then hold long runs of samples adding to one cell).  VISTA_AGGREGATE=0
// or 1 overrides the choice.
static int choose_aggregate(const HostLaunch& h) {
    if (const char* e = getenv("VISTA_AGGREGATE")) {
        if (e[0] == '0') return 0;
        if (e[0] == '1') return 1;
    }
    double fine = 0.0, all = 0.0;
    for (const HostTarget* ht : h.hts) {
        const double ns = (double)ht->t.nrow * ht->t.nchan * ht->t.npol;
        all += ns;
        if (ht->plan.chan_per_rest >= 6.0) fine += ns;
    }
    return all > 0.0 && fine >= 0.3 * all ? 1 : 0;
}

// Cells of one plane of a stack's carried state: every (tile, block) unit's full
// tu x tv x jc block, edge units included.
static int64_t carried_state_cells(const vista_grid_desc& g, const Tuning& tu) {
    const int64_t tiles = (int64_t)((g.nu + tu.tu - 1) / tu.tu) * ((g.nv + tu.tv - 1) / tu.tv);
    const int64_t nblocks = (g.nchan + tu.jc - 1) / tu.jc;
    return tiles * nblocks * tu.tu * tu.tv * tu.jc;
}

static HostLaunch build_launch(const std::vector<StackJob>& jobs, const Tuning& tu, int jsub) {
    {
        std::vector<HostTarget*> all;
        for (const StackJob& J : jobs) all.insert(all.end(), J.targets.begin(), J.targets.end());
        plan_all(all);
    }
    HostLaunch h;
    // The arena: the launch-wide channel tables (target i's entries start at its chan0),
    // then each target's block and in-band tables, every table 256-byte aligned.  Sized
    // first, then written in place.  The buffer is recycled, so only its growth is
    // zero-filled; padding between tables is never read.
    int64_t nch = 0, nfv = 0;
    size_t small = 0;
    for (const StackJob& J : jobs) {
        const int64_t nb = (J.g->nchan + tu.jc - 1) / tu.jc, nsb = (J.g->nchan + jsub - 1) / jsub;
        for (const HostTarget* ht : J.targets) {
            if (ht->t.nrow == 0) continue;
            nch += (int64_t)ht->plan.chan.size();
            nfv += (int64_t)ht->plan.fval.size();
            small += align256(2 * nb * sizeof(int32_t)) + align256((ht->plan.inband.size()) * sizeof(int32_t));
            if (jsub != tu.jc) small += align256(2 * nsb * sizeof(int32_t));
        }
    }
    if (nch >= 0x7fffffffLL || nfv >= 0x7fffffffLL) throw HipFail{hipErrorInvalidValue, "too many channels in one launch"};
    size_t cur = 0;
    auto take = [&cur](size_t n) {
        const size_t o = cur;
        cur = align256(cur + n);
        return o;
    };
    h.o_chan = take((size_t)nch * sizeof(DevChan));
    h.o_f1 = take((size_t)nch * sizeof(float));
    h.o_foff = take((size_t)nch * sizeof(int32_t));
    h.o_fval = take((size_t)nfv * sizeof(float));
    h.arena.swap(t_host.arena);
    h.arena.resize(std::max<size_t>(cur + small, 256));
    unsigned char* const A = h.arena.data();
    auto put = [&](const void* p, size_t n) {
        const size_t o = take(n);
        if (o + n > h.arena.size()) throw HipFail{hipErrorInvalidValue, "launch table sizes disagree"};
        if (n) memcpy(A + o, p, n);
        return o;
    };
    int64_t chan0 = 0, fval0 = 0;
    int64_t tiles = 0;
    h.dss.resize(jobs.size());
    for (size_t s = 0; s < jobs.size(); ++s) {
        const vista_grid_desc* g = jobs[s].g;
        DevStack& S = h.dss[s];
        memset(&S, 0, sizeof(S));
        S.nu = g->nu; S.nv = g->nv; S.nchan = g->nchan;
        S.tiles_u = (g->nu + tu.tu - 1) / tu.tu;
        S.tiles_v = (g->nv + tu.tv - 1) / tu.tv;
        S.nblocks = (g->nchan + tu.jc - 1) / tu.jc;
        S.inv_du = 1.0 / g->du;
        S.inv_dv = 1.0 / g->dv;
        S.target_begin = (int32_t)h.dts.size();
        S.tile_base = tiles;
        S.unit_base = h.nunits;
        S.out_vis = (float2*)jobs[s].out.sum_wvis;
        S.out_w = (float*)jobs[s].out.sum_w;
        S.out_cnt = (uint32_t*)jobs[s].out.count;
        S.out_vis64 = (double2*)jobs[s].out.sum_wvis64;
        S.out_w64 = (double*)jobs[s].out.sum_w64;
        S.st_s = jobs[s].st_s;
        S.st_c = jobs[s].st_c;
        S.st_n = jobs[s].st_n;
        S.st_plane = carried_state_cells(*g, tu);
        S.carry = jobs[s].carry;
        S.last = jobs[s].last;
        h.stats_index.push_back(jobs[s].index);
        h.tile_base.push_back(tiles);
        h.unit_base.push_back(h.nunits);
        tiles += (int64_t)S.tiles_u * S.tiles_v;
        h.nunits += (int64_t)S.tiles_u * S.tiles_v * S.nblocks;
        for (HostTarget* ht : jobs[s].targets) {
            if (ht->t.nrow == 0) continue;
            DevTarget T;
            memset(&T, 0, sizeof(T));
            T.row_base = h.rows;
            T.nrow = ht->t.nrow;
            T.nchan = ht->t.nchan;
            T.npol = ht->t.npol;
            T.weight_per_chan = ht->t.weight_per_chan;
            T.stack = (int32_t)s;
            T.kin_lo = ht->plan.kin_lo;
            T.kin_hi = ht->plan.kin_hi;
            T.nphase = ht->plan.nphase;
            T.nblocks = S.nblocks;
            T.l = ht->plan.frame.l; T.m = ht->plan.frame.m; T.nm1 = ht->plan.nm1;
            T.rotate = ht->plan.frame.rotate;
            for (int q = 0; q < 6; ++q) T.rot[q] = ht->plan.frame.R[q];
            T.chan0 = (int32_t)chan0;
            const size_t nc = ht->plan.chan.size();
            memcpy(A + h.o_chan + chan0 * sizeof(DevChan), ht->plan.chan.data(), nc * sizeof(DevChan));
            memcpy(A + h.o_f1 + chan0 * sizeof(float), ht->plan.f1.data(), nc * sizeof(float));
            int32_t* foff = (int32_t*)(A + h.o_foff) + chan0;
            for (size_t k = 0; k < nc; ++k) foff[k] = ht->plan.foff[k] + (int32_t)fval0;
            if (!ht->plan.fval.empty())
                memcpy(A + h.o_fval + fval0 * sizeof(float), ht->plan.fval.data(), ht->plan.fval.size() * sizeof(float));
            chan0 += (int64_t)nc;
            fval0 += (int64_t)ht->plan.fval.size();
            if (!ht->t.flag)
                h.zero_flag_bytes = std::max<int64_t>(h.zero_flag_bytes, (int64_t)ht->t.nchan * ht->t.npol);
            if (T.npol != 2 || T.weight_per_chan) h.npol_all = 0;   // the specialised path: 2 pols, row weights
            HostLaunch::Offs o;
            std::vector<int32_t> blk = block_ranges(ht->plan, g->nchan, tu.jc);
            o.blk = put(blk.data(), blk.size() * sizeof(int32_t));
            if (jsub != tu.jc) {
                std::vector<int32_t> sblk = block_ranges(ht->plan, g->nchan, jsub);
                o.sblk = put(sblk.data(), sblk.size() * sizeof(int32_t));
            } else {
                o.sblk = o.blk;
            }
            o.inband = put(ht->plan.inband.data(), ht->plan.inband.size() * sizeof(int32_t));
            h.offs.push_back(o);
            h.row_base.push_back(h.rows);
            h.rows += ht->t.nrow;
            h.dts.push_back(T);
            h.hts.push_back(ht);
        }
        S.target_end = (int32_t)h.dts.size();
    }
    h.row_base.push_back(h.rows);
    h.tile_base.push_back(tiles);
    h.unit_base.push_back(h.nunits);
    h.agg = choose_aggregate(h);
    // One thread per row, unit or record in the element-wise passes: a dispatch's work-item
    // count is 32 bits wide, so each count stays below 2^32 - 256 (a whole last block).
    if (h.rows >= kMaxItems) throw HipFail{hipErrorInvalidValue, "2^32-256 rows or more in one launch"};
    if (h.nunits >= kMaxItems) throw HipFail{hipErrorInvalidValue, "too many (tile, block) units in one launch"};
    h.arena.resize(std::max<size_t>(cur, 256));
    return h;
}

// Sizes of the fixed device buffers of the launch sequence.
struct Capacity {
    int64_t rows = 0, targets = 0, stacks = 0, arena = 0, units = 0, recs = 0, zflag = 0;
    static Capacity of(const HostLaunch& h) {
        Capacity c;
        c.rows = h.rows;
        c.targets = (int64_t)h.dts.size();
        c.stacks = (int64_t)h.dss.size();
        c.arena = (int64_t)h.arena.size();
        c.units = h.nunits;
        c.zflag = h.zero_flag_bytes;
        return c;
    }
    Capacity max_with(const Capacity& o) const {
        Capacity c;
        c.rows = std::max(rows, o.rows); c.targets = std::max(targets, o.targets);
        c.stacks = std::max(stacks, o.stacks); c.arena = std::max(arena, o.arena);
        c.units = std::max(units, o.units); c.recs = std::max(recs, o.recs); c.zflag = std::max(zflag, o.zflag);
        return c;
    }
    bool covers(const Capacity& o) const {
        return rows >= o.rows && targets >= o.targets && stacks >= o.stacks && arena >= o.arena &&
               units >= o.units && recs >= o.recs && zflag >= o.zflag;
    }
};

// The device side of launches: fixed buffers sized by a capacity, the count pass (run
// eagerly, it sizes the record buffers), and the rest of the sequence -- emit, sort, unit
// offsets, record starts, work list, accumulation -- which reads every count from device
// memory, records no memset and never synchronises, so it can be captured once in a
// hipGraph and replayed for every launch that fits the capacity.
class Launcher {
  public:
    Launcher(hipStream_t s, const Tuning& tu, uint32_t flags, bool persistent = false)
        : s_(s), tu_(tu), mem_(s, persistent), recmem_(s, persistent) {
        mode_ = (flags & VISTA_F_DETERMINISTIC) ? kModeOrdered : kModeAtomic;
        kahan_ = (flags & VISTA_F_KAHAN) ? 1 : 0;
        acc32_ = (flags & VISTA_F_PLAIN_FP32) ? 1 : 0;
        phase_fp32_ = (flags & VISTA_F_PHASE_FP32) ? 1 : 0;
        jsub_ = mode_ == kModeOrdered ? tu.jc / tu.waves : tu.jc;
        if (!shape_ok(tu, flags)) throw HipFail{hipErrorInvalidValue, "unsupported launch shape (tile/jblock/waves)"};
    }
    ~Launcher() { drop_graph(); }
    // Launch on another stream (a cached launcher between calls; no graph is captured then).
    void set_stream(hipStream_t s) {
        s_ = s;
        mem_.set_stream(s);
        recmem_.set_stream(s);
    }
    int jsub() const { return jsub_; }

    // Grow the buffers to cover c (record buffers separately: they are sized last).
    void reserve(const Capacity& want) {
        Capacity c = cap_.max_with(want);
        if (!cap_.covers(Capacity{c.rows, c.targets, c.stacks, c.arena, c.units, 0, c.zflag}) || !fixed_) {
            drop_graph();
            mem_.release();
            fixed_ = true;
            d_L_ = mem_.alloc_n<LaunchDesc>(1);
            d_t_ = mem_.alloc_n<DevTarget>(std::max<int64_t>(1, c.targets));
            d_s_ = mem_.alloc_n<DevStack>(std::max<int64_t>(1, c.stacks));
            d_rb_ = mem_.alloc_n<int64_t>(c.targets + 1);
            d_tb_ = mem_.alloc_n<int64_t>(c.stacks + 1);
            d_ub_ = mem_.alloc_n<int64_t>(c.stacks + 1);
            d_arena_ = mem_.alloc_n<unsigned char>(std::max<int64_t>(256, c.arena));
            rowctx_ = mem_.alloc_n<RowCtx>(std::max<int64_t>(1, c.rows));
            row_target_ = mode_ == kModeOrdered ? mem_.alloc_n<int32_t>(std::max<int64_t>(1, c.rows)) : nullptr;
            zflags_ = nullptr;
            if (c.zflag > 0) {
                int64_t words = (c.zflag + 3) / 4;
                uint32_t* z = mem_.alloc_n<uint32_t>(words);
                check_launch(launch_fill_u32(z, 0u, words, s_), "fill");
                zflags_ = (const uint8_t*)z;
            }
            cnt_ = mem_.alloc_n<uint32_t>(std::max<int64_t>(1, c.rows));
            off_ = mem_.alloc_n<uint32_t>(c.rows + 1);
            sums_ = mem_.alloc_n<uint64_t>(scan_temp_elems(c.rows));
            unit_off_ = mem_.alloc_n<uint32_t>(c.units + 1);
            okeys_ = mem_.alloc_n<uint32_t>(std::max<int64_t>(1, c.units));
            order_ = mem_.alloc_n<uint64_t>(std::max<int64_t>(1, c.units));
            otmp_ = mem_.alloc(radix_sort_temp_bytes(std::max<int64_t>(1, c.units)));
            counter_ = mem_.alloc_n<uint32_t>(1);
            cap_ = Capacity{c.rows, c.targets, c.stacks, c.arena, c.units, cap_.recs, c.zflag};
            recs_ok_ = false;
        }
        if (!recs_ok_ || want.recs > cap_.recs) {
            drop_graph();
            recmem_.release();
            const int64_t r = std::max<int64_t>(std::max(want.recs, cap_.recs), 1);
            keys_ = recmem_.alloc_n<uint32_t>(r);
            vals_ = recmem_.alloc_n<uint64_t>(r);
            stmp_ = recmem_.alloc(radix_sort_temp_bytes(r));
            lens_ = recmem_.alloc_n<uint32_t>(r);
            pre_ = recmem_.alloc_n<uint64_t>(r + 1);
            psums_ = recmem_.alloc_n<uint64_t>(scan_temp_elems(r));
            cap_.recs = r;
            recs_ok_ = true;
        }
    }

    // Upload launch h into the fixed buffers and run the count pass (which also writes
    // the row contexts and the outside-uv counts).  Returns the number of records.
    int64_t prepare(HostLaunch& h, unsigned long long* d_stats) {
        if (!cap_.covers(Capacity::of(h)) || !fixed_) throw HipFail{hipErrorInvalidValue, "launch exceeds capacity"};
        const DevChan* d_chan = (const DevChan*)(d_arena_ + h.o_chan);
        const float* d_f1 = (const float*)(d_arena_ + h.o_f1);
        const int32_t* d_foff = (const int32_t*)(d_arena_ + h.o_foff);
        const float* d_fval = (const float*)(d_arena_ + h.o_fval);
        for (size_t i = 0; i < h.dts.size(); ++i) {
            DevTarget& T = h.dts[i];
            T.chan = d_chan + T.chan0;
            T.f1 = d_f1 + T.chan0;
            T.foff = d_foff + T.chan0;
            T.fval = d_fval;
            T.blk = (const int32_t*)(d_arena_ + h.offs[i].blk);
            T.sblk = (const int32_t*)(d_arena_ + h.offs[i].sblk);
            T.inband = (const int32_t*)(d_arena_ + h.offs[i].inband);
        }
        for (size_t s = 0; s < h.dss.size(); ++s) h.dss[s].stats = d_stats + 8 * h.stats_index[s];
        LaunchDesc& L = L_;
        memset(&L, 0, sizeof(L));
        L.targets = d_t_;
        L.stacks = d_s_;
        L.target_row_base = d_rb_;
        L.stack_tile_base = d_tb_;
        L.stack_unit_base = d_ub_;
        L.ntargets = (int32_t)h.dts.size();
        L.nstacks = (int32_t)h.dss.size();
        L.tu = tu_.tu; L.tv = tu_.tv; L.jc = tu_.jc; L.jsub = jsub_;
        L.nrows = h.rows;
        L.mode = mode_;
        L.kahan = kahan_;
        L.phase_fp32 = phase_fp32_;
        L.nunits = h.nunits;
        L.chan_all = d_chan;
        L.f1_all = d_f1;
        L.foff_all = d_foff;
        L.fval_all = d_fval;
        L.rowctx = rowctx_;
        L.row_target = row_target_;
        L.zero_flags = zflags_;
        npol_ = h.npol_all;
        agg_ = h.agg;
        // host sources stay alive until the stream has passed these copies (the count
        // below synchronises)
        VISTA_HIP(hipMemcpyAsync(d_arena_, h.arena.data(), h.arena.size(), hipMemcpyHostToDevice, s_));
        if (!h.dts.empty())
            VISTA_HIP(hipMemcpyAsync(d_t_, h.dts.data(), h.dts.size() * sizeof(DevTarget), hipMemcpyHostToDevice, s_));
        VISTA_HIP(hipMemcpyAsync(d_s_, h.dss.data(), h.dss.size() * sizeof(DevStack), hipMemcpyHostToDevice, s_));
        VISTA_HIP(hipMemcpyAsync(d_rb_, h.row_base.data(), h.row_base.size() * 8, hipMemcpyHostToDevice, s_));
        VISTA_HIP(hipMemcpyAsync(d_tb_, h.tile_base.data(), h.tile_base.size() * 8, hipMemcpyHostToDevice, s_));
        VISTA_HIP(hipMemcpyAsync(d_ub_, h.unit_base.data(), h.unit_base.size() * 8, hipMemcpyHostToDevice, s_));
        VISTA_HIP(hipMemcpyAsync(d_L_, &L, sizeof(L), hipMemcpyHostToDevice, s_));
        // count pass: records per row, their exclusive scan (total at the scan's end slot)
        check_launch(launch_track(cap_.rows, d_L_, cnt_, nullptr, nullptr, nullptr, 0, s_), "track count");
        check_launch(exclusive_scan_u32_to_u32(cnt_, nrows_dev(), cap_.rows, off_, sums_, s_), "scan");
        uint64_t total = 0;
        VISTA_HIP(hipMemcpyAsync(&total, nrec_dev(), 8, hipMemcpyDeviceToHost, s_));
        VISTA_HIP(hipStreamSynchronize(s_));
        if (total >= (uint64_t)kMaxItems) throw HipFail{hipErrorInvalidValue, "too many track records in one launch"};
        return (int64_t)total;
    }

    // The rest of the sequence for the uploaded launch.  ev (optional, eager only) gets
    // its events 1 and 2 around the accumulation.
    void sequence(Events* ev) {
        binning();
        if (ev) VISTA_HIP(hipEventRecord(ev->e[1], s_));
        accumulate();
        if (ev) VISTA_HIP(hipEventRecord(ev->e[2], s_));
    }

    // Replay the captured binning part (capturing it first, or again after the buffers
    // changed), then launch the accumulation itself; `mid` (optional)
    // is recorded between the two, so that the accumulation kernel is timed on its own.
    void replay(hipEvent_t mid) {
        if (!exec_) {
            drop_graph();
            VISTA_HIP(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal));
            try {
                binning();
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(s_, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            VISTA_HIP(hipStreamEndCapture(s_, &graph_));
            VISTA_HIP(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
            ++captures_;
        }
        VISTA_HIP(hipGraphLaunch(exec_, s_));
        if (mid) VISTA_HIP(hipEventRecord(mid, s_));
        accumulate();
    }
    int captures() const { return captures_; }
    const Capacity& capacity() const { return cap_; }

  private:
    // After the count pass: emit the records, sort them by unit, unit offsets, record
    // prefix sums, the units' work order, the work counter cleared.  Every size it needs is
    // read from device memory, and it records no memset, so that a graph can hold it.
    void binning() {
        check_launch(launch_track(cap_.rows, d_L_, nullptr, off_, keys_, vals_, 1, s_), "track emit");
        int bits = 1;
        while (bits < 32 && (int64_t(1) << bits) < cap_.units) ++bits;
        check_launch(radix_sort_pairs(keys_, vals_, nrec_dev(), cap_.recs, bits, stmp_, s_), "sort");
        check_launch(launch_unit_offsets(keys_, nrec_dev(), cap_.recs, nunits_dev(), cap_.units, unit_off_, s_), "unit offsets");
        check_launch(launch_record_prefix(vals_, nrec_dev(), cap_.recs, lens_, pre_, psums_, s_), "record prefix");
        check_launch(launch_unit_order(d_L_, unit_off_, pre_, nunits_dev(), cap_.units, okeys_, order_, otmp_, s_),
                     "unit order");
        check_launch(launch_fill_u32(counter_, 0u, 1, s_), "fill");
    }

    // The accumulation kernel over the work list, one persistent grid.
    void accumulate() {
        int per_cu = tu_.wg_per_cu;
        if (per_cu <= 0)
            per_cu = mode_ == kModeAtomic
                         ? accum_packed_max_blocks_per_cu(tu_.tu, tu_.tv, tu_.jc, tu_.waves, npol_, acc32_, agg_)
                         : accum_max_blocks_per_cu(tu_.tu, tu_.tv, tu_.jc, tu_.waves, mode_, kahan_, npol_);
        if (per_cu < 1) per_cu = 1;
        const int64_t grid = std::min<int64_t>((int64_t)per_cu * device_cus(), std::max<int64_t>(1, cap_.units));
        if (mode_ == kModeAtomic)
            check_launch(launch_accum_packed(L_, d_L_, order_, counter_, unit_off_, vals_, pre_, (int)grid, tu_.waves,
                                             npol_, acc32_, agg_, s_),
                         "accumulate");
        else
            check_launch(launch_accum_impl(L_, d_L_, order_, counter_, unit_off_, vals_, (int)grid, tu_.waves, npol_,
                                           s_),
                         "accumulate");
    }
    const int64_t* nrows_dev() const { return (const int64_t*)((const char*)d_L_ + offsetof(LaunchDesc, nrows)); }
    const int64_t* nunits_dev() const { return (const int64_t*)((const char*)d_L_ + offsetof(LaunchDesc, nunits)); }
    const int64_t* nrec_dev() const { return (const int64_t*)(sums_ + (scan_temp_elems(cap_.rows) - 1)); }
    void drop_graph() {
        if (exec_) (void)hipGraphExecDestroy(exec_);
        if (graph_) (void)hipGraphDestroy(graph_);
        exec_ = nullptr;
        graph_ = nullptr;
    }

    hipStream_t s_;
    Tuning tu_;
    int mode_ = kModeAtomic, kahan_ = 0, acc32_ = 0, phase_fp32_ = 0, jsub_ = 0, npol_ = 2, agg_ = 0;
    DevMem mem_, recmem_;
    Capacity cap_;
    bool fixed_ = false, recs_ok_ = false;
    LaunchDesc L_{};
    LaunchDesc* d_L_ = nullptr;
    DevTarget* d_t_ = nullptr;
    DevStack* d_s_ = nullptr;
    int64_t *d_rb_ = nullptr, *d_tb_ = nullptr, *d_ub_ = nullptr;
    unsigned char* d_arena_ = nullptr;
    RowCtx* rowctx_ = nullptr;
    int32_t* row_target_ = nullptr;
    const uint8_t* zflags_ = nullptr;
    uint32_t *cnt_ = nullptr, *off_ = nullptr, *unit_off_ = nullptr, *okeys_ = nullptr, *counter_ = nullptr;
    uint64_t *sums_ = nullptr, *order_ = nullptr;
    void* otmp_ = nullptr;
    uint32_t* keys_ = nullptr;
    uint64_t* vals_ = nullptr;
    void* stmp_ = nullptr;
    uint32_t* lens_ = nullptr;
    uint64_t *pre_ = nullptr, *psums_ = nullptr;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
    int captures_ = 0;
};

// Point the launch's targets at device copies of their data: device-resident inputs as
// they are, host inputs copied into `mem` (stream-ordered on s).
static void make_resident(HostLaunch& h, DevMem& mem, hipStream_t s) {
    for (size_t i = 0; i < h.dts.size(); ++i) {
        DevTarget& T = h.dts[i];
        const vista_target& t = h.hts[i]->t;
        if (t.mem == VISTA_MEM_DEVICE) {
            T.uvw = t.uvw; T.vis = (const float2*)t.vis; T.weight = t.weight; T.flag = t.flag;
            continue;
        }
        size_t nr = (size_t)t.nrow, ns = nr * t.nchan * t.npol;
        size_t b_w = (t.weight_per_chan ? ns : nr * t.npol) * sizeof(float);
        double* du = mem.alloc_n<double>(nr * 3);
        float2* dv = mem.alloc_n<float2>(ns);
        float* dw = (float*)mem.alloc(b_w);
        VISTA_HIP(hipMemcpyAsync(du, t.uvw, nr * 3 * sizeof(double), hipMemcpyHostToDevice, s));
        VISTA_HIP(hipMemcpyAsync(dv, t.vis, ns * 8, hipMemcpyHostToDevice, s));
        VISTA_HIP(hipMemcpyAsync(dw, t.weight, b_w, hipMemcpyHostToDevice, s));
        T.uvw = du; T.vis = dv; T.weight = dw; T.flag = nullptr;
        if (t.flag) {
            uint8_t* df = mem.alloc_n<uint8_t>(ns);
            VISTA_HIP(hipMemcpyAsync(df, t.flag, ns, hipMemcpyHostToDevice, s));
            T.flag = df;
        }
    }
}

static void collect_stats(std::vector<StackJob>& jobs, const std::vector<unsigned long long>& st) {
    for (size_t s = 0; s < jobs.size(); ++s) {
        vista_stats& o = jobs[s].stats;
        memset(&o, 0, sizeof(o));
        for (HostTarget* h : jobs[s].targets) {
            o.n_samples += h->n_samples;
            o.n_outside_band += h->n_outside_band;
        }
        const size_t k = 8 * (size_t)jobs[s].index;
        o.n_flagged = st[k + 1];
        o.n_bad_weight = st[k + 2];
        o.n_outside_uv = st[k + 3];
        o.n_used = st[k + 5];
        o.n_contrib = st[k + 6];
        jobs[s].overflow = st[k + 7];
    }
}

// Stack every job in one eager pass (the plain form: one launch sequence).  All output
// cells of every job are written.
// A thread's launch workspaces: the launcher (its fixed and record buffers grow to the
// largest launch seen and are then reused), events and a statistics buffer, per device,
// launch shape and accumulation mode, so that consecutive stacks neither allocate nor free
// device memory.  At most two are kept (the autotuner cycles through shapes); they are
// freed by vista_release_workspace, or when evicted.
struct Workspace {
    int device = 0;
    Tuning tu;
    uint32_t mode_flags = 0;
    std::unique_ptr<Launcher> ln;
    std::unique_ptr<Events> ev;
    std::unique_ptr<DevMem> stats_mem;
    unsigned long long* stats = nullptr;
    size_t stats_cap = 0;
    unsigned long long* stats_for(size_t n) {
        if (n > stats_cap) {
            stats_mem->release();
            stats_cap = std::max<size_t>(n, 64);
            stats = stats_mem->alloc_n<unsigned long long>(stats_cap);
        }
        return stats;
    }
};
static thread_local std::vector<std::unique_ptr<Workspace>> t_workspaces;
constexpr size_t kMaxWorkspaces = 2;

static Workspace& workspace_for(hipStream_t stream, const Tuning& tu, uint32_t flags) {
    int dev = 0;
    VISTA_HIP(hipGetDevice(&dev));
    const uint32_t mf = flags & (VISTA_F_DETERMINISTIC | VISTA_F_KAHAN | VISTA_F_PHASE_FP32 | VISTA_F_PLAIN_FP32);
    for (size_t i = 0; i < t_workspaces.size(); ++i) {
        Workspace& w = *t_workspaces[i];
        if (w.device == dev && w.mode_flags == mf && w.tu.tu == tu.tu && w.tu.tv == tu.tv && w.tu.jc == tu.jc &&
            w.tu.waves == tu.waves && w.tu.wg_per_cu == tu.wg_per_cu) {
            std::unique_ptr<Workspace> keep = std::move(t_workspaces[i]);     // most recent last
            t_workspaces.erase(t_workspaces.begin() + i);
            t_workspaces.push_back(std::move(keep));
            t_workspaces.back()->ln->set_stream(stream);
            return *t_workspaces.back();
        }
    }
    if (t_workspaces.size() >= kMaxWorkspaces) t_workspaces.erase(t_workspaces.begin());
    auto w = std::make_unique<Workspace>();
    w->device = dev;
    w->tu = tu;
    w->mode_flags = mf;
    w->ln = std::make_unique<Launcher>(stream, tu, flags, true);
    w->ev = std::make_unique<Events>();
    w->stats_mem = std::make_unique<DevMem>(stream, true);
    t_workspaces.push_back(std::move(w));
    return *t_workspaces.back();
}

// Drop the workspace of (tu, flags) after a failure: its buffers' contents are unknown.
static void drop_workspace(const Workspace* w) {
    for (size_t i = 0; i < t_workspaces.size(); ++i)
        if (t_workspaces[i].get() == w) {
            t_workspaces.erase(t_workspaces.begin() + i);
            return;
        }
}

static void run_jobs_in(Workspace& ws, std::vector<StackJob>& jobs, const Tuning& tu, hipStream_t stream,
                        vista_timings* tim);

static void run_jobs(std::vector<StackJob>& jobs, const Tuning& tu, uint32_t flags, hipStream_t stream,
                     vista_timings* tim) {
    Workspace& ws = workspace_for(stream, tu, flags);
    try {
        run_jobs_in(ws, jobs, tu, stream, tim);
    } catch (...) {
        drop_workspace(&ws);
        throw;
    }
}

static void run_jobs_in(Workspace& ws, std::vector<StackJob>& jobs, const Tuning& tu, hipStream_t stream,
                        vista_timings* tim) {
    DevMem mem(stream);                   // staging of host-memory targets only
    Events& ev = *ws.ev;
    Launcher& ln = *ws.ln;
    for (size_t s = 0; s < jobs.size(); ++s) jobs[s].index = (int32_t)s;
    HostLaunch h = build_launch(jobs, tu, ln.jsub());
    VISTA_HIP(hipEventRecord(ev.e[0], stream));
    make_resident(h, mem, stream);
    unsigned long long* d_stats = ws.stats_for(8 * jobs.size());
    check_launch(launch_fill_u64(d_stats, 0ull, 8 * (int64_t)jobs.size(), stream), "fill");
    ln.reserve(Capacity::of(h));
    const int64_t nrec = ln.prepare(h, d_stats);
    Capacity c = Capacity::of(h);
    c.recs = nrec;
    ln.reserve(c);
    ln.sequence(&ev);
    std::vector<unsigned long long> st(8 * jobs.size());
    VISTA_HIP(hipMemcpyAsync(st.data(), d_stats, st.size() * 8, hipMemcpyDeviceToHost, stream));
    VISTA_HIP(hipEventRecord(ev.e[3], stream));
    VISTA_HIP(hipStreamSynchronize(stream));
    collect_stats(jobs, st);
    vlog(1, "stack launch: %zu stack(s), %zu target(s), %lld rows, %lld records, %lld units, shape %dx%dx%d/%d%s; "
            "binning %.3f ms, accumulation %.3f ms, total %.3f ms",
         jobs.size(), h.dts.size(), (long long)h.rows, (long long)nrec, (long long)h.nunits, tu.tu, tu.tv, tu.jc,
         tu.waves, h.agg ? " aggregated" : "", ev.ms(0, 1), ev.ms(1, 2), ev.ms(0, 3));
    if (tim) {
        tim->bin_ms = ev.ms(0, 1);
        tim->accum_ms = ev.ms(1, 2);
        tim->finalize_ms = ev.ms(2, 3);
        tim->total_ms = ev.ms(0, 3);
        tim->h2d_ms = 0;
        tim->n_records = nrec;
        tim->n_units = h.nunits;
        tim->n_accum_launches = 1;
        tim->n_waves = 1;
    }
}

// ------------------------------------------------------------------------ autotuning

// Candidate launch shapes of a mode: every (tile, block) shape the kernel is built for.
// The packed kernel's come with 16 wavefronts per workgroup, and with 8 where two
// workgroups share a compute unit's LDS.  The ordered kernel's come with the fewest
// wavefronts (1, 2, 4, 8 or 16) whose workgroups, 16 wavefronts' worth, fit one compute
// unit's LDS: every wavefront of a workgroup walks all of its unit's records, so fewer per
// workgroup walk less at the same occupancy.  The first candidate is the mode's default.
static std::vector<Tuning> tuning_candidates(uint32_t flags) {
    const int mode = (flags & VISTA_F_DETERMINISTIC) ? kModeOrdered : kModeAtomic;
    const int kahan = (flags & VISTA_F_KAHAN) ? 1 : 0;
    const int acc32 = (flags & VISTA_F_PLAIN_FP32) ? 1 : 0;
    int tu[64], tv[64], jc[64];
    const int n = std::min(mode == kModeAtomic ? accum_packed_shape_list(acc32, tu, tv, jc, 64)
                                               : accum_shape_list(mode, tu, tv, jc, 64),
                           64);
    std::vector<Tuning> out{default_tuning(flags)};
    for (int i = 0; i < n; ++i) {
        if (mode == kModeOrdered) {
            const size_t lds = accum_lds_bytes(tu[i], tv[i], jc[i], mode, kahan);
            for (int waves : {1, 2, 4, 8, 16}) {
                Tuning t;
                t.tu = tu[i]; t.tv = tv[i]; t.jc = jc[i]; t.waves = waves;
                if (lds * (16 / waves) > 160 * 1024 || !shape_ok(t, flags)) continue;
                if (!(t.tu == out[0].tu && t.tv == out[0].tv && t.jc == out[0].jc && t.waves == out[0].waves))
                    out.push_back(t);
                break;
            }
            continue;
        }
        for (int waves : {16, 8}) {
            Tuning t;
            t.tu = tu[i]; t.tv = tv[i]; t.jc = jc[i]; t.waves = waves;
            if (!shape_ok(t, flags)) continue;
            if (waves == 8 && accum_packed_lds_bytes(t.tu, t.tv, t.jc, acc32) > 80 * 1024) continue;
            if (t.tu == out[0].tu && t.tv == out[0].tv && t.jc == out[0].jc && t.waves == out[0].waves) continue;
            out.push_back(t);
        }
    }
    return out;
}

// Time every candidate shape on the jobs (device-resident targets; each job's outputs are
// scratch buffers with a count grid) and return the fastest whose count grids equal the
// default shape's bit for bit.  reps runs per candidate, the median time counts.
static Tuning autotune_jobs(std::vector<StackJob>& jobs, uint32_t flags, hipStream_t stream, int reps,
                            double* best_ms) {
    DevMem mem(stream);
    std::vector<uint32_t*> ref(jobs.size());
    std::vector<int64_t> ncell(jobs.size());
    for (size_t j = 0; j < jobs.size(); ++j) {
        const vista_grid_desc* g = jobs[j].g;
        ncell[j] = (int64_t)g->nu * g->nv * g->nchan;
        ref[j] = mem.alloc_n<uint32_t>(ncell[j]);
    }
    uint32_t* flag = mem.alloc_n<uint32_t>(1);
    std::vector<Tuning> cand = tuning_candidates(flags);
    Tuning best = cand[0];
    double best_t = 1e300;
    for (size_t c = 0; c < cand.size(); ++c) {
        std::vector<double> ts;
        for (int r = 0; r < std::max(1, reps); ++r) {
            vista_timings tim{};
            run_jobs(jobs, cand[c], flags, stream, &tim);
            ts.push_back(tim.total_ms);
        }
        std::sort(ts.begin(), ts.end());
        const double t = ts[ts.size() / 2];
        bool same = true;
        if (c == 0) {
            for (size_t j = 0; j < jobs.size(); ++j)
                VISTA_HIP(hipMemcpyAsync(ref[j], jobs[j].out.count, ncell[j] * 4, hipMemcpyDeviceToDevice, stream));
        } else {
            check_launch(launch_fill_u32(flag, 0u, 1, stream), "fill");
            for (size_t j = 0; j < jobs.size(); ++j)
                check_launch(launch_diff_u32(ref[j], (const uint32_t*)jobs[j].out.count, ncell[j], flag, stream),
                             "compare");
            uint32_t h = 0;
            VISTA_HIP(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, stream));
            VISTA_HIP(hipStreamSynchronize(stream));
            same = h == 0;
        }
        vlog(2, "autotune candidate %dx%dx%d/%d: %.3f ms%s", cand[c].tu, cand[c].tv, cand[c].jc, cand[c].waves, t,
             same ? "" : " (counts differ from the default shape: rejected)");
        if (same && t < best_t) {
            best_t = t;
            best = cand[c];
        }
    }
    VISTA_HIP(hipStreamSynchronize(stream));
    if (best_ms) *best_ms = best_t;
    return best;
}

// ------------------------------------------------------------------ tuning cache

// VISTA_TUNE_CACHE names a file of JSON lines, one per tuned workload:
//   {"key": "<16 hex digits>", "tile_u": 8, "tile_v": 4, "jblock": 160, "waves": 16, "ms": 31.2,
//    "workload": "<the signature hashed into key>"}
// The signature holds the device's architecture and compute units, the accumulation flags,
// every stack's grid shape and its targets' count, rows, channels and samples.  An autotune
// call whose key is in the file takes that shape without timing anything (if the shape is
// still built and valid for the flags); otherwise it times the candidates and appends the
// winner.  Lines that do not parse are ignored.
static std::string tune_signature(const std::vector<StackJob>& jobs, uint32_t flags) {
    std::string sig;
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
        sig += std::string(p.gcnArchName) + "/" + std::to_string(p.multiProcessorCount);
    sig += " flags=" + std::to_string(flags & (VISTA_F_KAHAN | VISTA_F_DETERMINISTIC | VISTA_F_PHASE_FP32 |
                                               VISTA_F_PLAIN_FP32 | VISTA_F_SPECTRAL_NEAREST));
    for (const StackJob& J : jobs) {
        int64_t rows = 0, chans = 0, samples = 0;
        int npol_mask = 0;
        for (const HostTarget* h : J.targets) {
            rows += h->t.nrow;
            chans += h->t.nchan;
            samples += h->t.nrow * (int64_t)h->t.nchan * h->t.npol;
            npol_mask |= 1 << h->t.npol | (h->t.weight_per_chan ? 32 : 0);
        }
        sig += " " + std::to_string(J.g->nu) + "x" + std::to_string(J.g->nv) + "x" + std::to_string(J.g->nchan) + ":" +
               std::to_string(J.targets.size()) + "/" + std::to_string(rows) + "/" + std::to_string(chans) + "/" +
               std::to_string(samples) + "/" + std::to_string(npol_mask);
    }
    return sig;
}

static std::string tune_key(const std::string& sig) {
    uint64_t h = 1469598103934665603ull;            // FNV-1a, 64 bit
    for (unsigned char c : sig) {
        h ^= c;
        h *= 1099511628211ull;
    }
    char buf[17];
    snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
    return buf;
}

static bool tune_cache_lookup(const std::string& key, uint32_t flags, Tuning* out) {
    const char* path = getenv("VISTA_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[4096];
    bool found = false;
    const std::string want = "\"key\": \"" + key + "\"";
    while (fgets(line, sizeof(line), f)) {
        if (!strstr(line, want.c_str())) continue;
        auto field = [&](const char* name, int* v) {
            const char* q = strstr(line, name);
            if (!q) return false;
            q += strlen(name);
            while (*q == ' ' || *q == ':') ++q;
            char* end = nullptr;
            const long x = strtol(q, &end, 10);
            if (end == q || x < 1 || x > 100000) return false;
            *v = (int)x;
            return true;
        };
        Tuning t;
        if (field("\"tile_u\"", &t.tu) && field("\"tile_v\"", &t.tv) && field("\"jblock\"", &t.jc) &&
            field("\"waves\"", &t.waves) && shape_ok(t, flags)) {
            *out = t;                                  // the last valid line for the key wins
            found = true;
        }
    }
    fclose(f);
    return found;
}

static void tune_cache_store(const std::string& key, const std::string& sig, const Tuning& t, double ms) {
    const char* path = getenv("VISTA_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "a");
    if (!f) {
        vlog(1, "tuning cache %s cannot be opened for appending", path);
        return;
    }
    fprintf(f, "{\"key\": \"%s\", \"tile_u\": %d, \"tile_v\": %d, \"jblock\": %d, \"waves\": %d, \"ms\": %.4f, "
               "\"workload\": \"%s\"}\n",
            key.c_str(), t.tu, t.tv, t.jc, t.waves, ms, sig.c_str());
    fclose(f);
}

// The autotuner behind the cache; `prepare` (scratch outputs for the timed runs) is called
// only when the shape must be timed.
template <class F>
static Tuning autotune_cached(std::vector<StackJob>& jobs, uint32_t flags, hipStream_t stream, bool* from_cache,
                              F&& prepare) {
    const std::string sig = tune_signature(jobs, flags);
    const std::string key = tune_key(sig);
    Tuning t;
    if (tune_cache_lookup(key, flags, &t)) {
        vlog(2, "autotune: shape %dx%dx%d/%d from the tuning cache (key %s)", t.tu, t.tv, t.jc, t.waves, key.c_str());
        *from_cache = true;
        return t;
    }
    prepare();
    double ms = 0;
    t = autotune_jobs(jobs, flags, stream, 2, &ms);
    tune_cache_store(key, sig, t, ms);
    *from_cache = false;
    return t;
}

// Scratch outputs (sum_wvis, sum_w, count) of one job, for autotuning.
static void scratch_outputs(StackJob& J, DevMem& mem) {
    const size_t nc = (size_t)J.g->nu * J.g->nv * J.g->nchan;
    J.out = vista_output{};
    J.out.sum_wvis = mem.alloc(nc * 8);
    J.out.sum_w = mem.alloc(nc * 4);
    J.out.count = mem.alloc(nc * 4);
    J.out.mem = VISTA_MEM_DEVICE;
}

static void to_public(const Tuning& t, vista_tuning* o) {
    if (!o) return;
    o->tile_u = t.tu; o->tile_v = t.tv; o->jblock = t.jc; o->waves = t.waves; o->wg_per_cu = t.wg_per_cu;
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

int vista_release_workspace(void) {
    return guarded(nullptr, [&]() -> int {
        t_workspaces.clear();
        t_host = HostScratch();
        g_dev_bytes -= BigBlocks::get().release(current_device());
        return VISTA_OK;
    });
}

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
        if (h->planned && !check_plan(h->plan, &w)) return fail(VISTA_E_ARG, w);
        s->targets.reserve(s->targets.size() + 1);
        plan_in_background(h.get());
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
        if (jobs[0].overflow) return fault_fail(jobs[0].overflow);
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
        copy_target(h, g, t, true);
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
        T.rotate = h.plan.frame.rotate;
        for (int q = 0; q < 6; ++q) T.rot[q] = h.plan.frame.R[q];
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
        copy_target(h, g, t, true);
        DevMem mem(stream);
        DevChan* dch = mem.alloc_n<DevChan>(t->nchan);
        VISTA_HIP(hipMemcpyAsync(dch, h.plan.chan.data(), t->nchan * sizeof(DevChan), hipMemcpyHostToDevice, stream));
        DevTarget T;
        memset(&T, 0, sizeof(T));
        T.uvw = t->uvw; T.vis = (const float2*)t->vis; T.chan = dch; T.nrow = t->nrow; T.nchan = t->nchan;
        T.npol = t->npol; T.l = h.plan.frame.l; T.m = h.plan.frame.m; T.nm1 = h.plan.nm1;
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

// ------------------------------------------------------------------ rebinned rows

static bool check_rebin_desc(const vista_rebin_desc* d, std::string* why) {
    if (!d) { *why = "rebin descriptor is NULL"; return false; }
    if (d->nout < 1 || d->nout > (1 << 20)) { *why = "nout must be in 1..1048576"; return false; }
    if (!(d->dfreq > 0 && std::isfinite(d->dfreq))) { *why = "dfreq must be finite and > 0"; return false; }
    if (!std::isfinite(d->central_freq)) { *why = "central_freq must be finite"; return false; }
    return true;
}

// The channel axis of a target (what the window and the tables read).
static bool check_channels(const vista_target* t, std::string* why) {
    if (!t) { *why = "target is NULL"; return false; }
    vista_target c = *t;
    c.nrow = 0;
    return check_target(nullptr, &c, why);
}

int vista_rebin_window(const vista_rebin_desc* d, const vista_target* t, double* freq_lo) {
    std::string why;
    if (!check_rebin_desc(d, &why) || !check_channels(t, &why)) return fail(VISTA_E_ARG, why);
    if (!freq_lo) return fail(VISTA_E_ARG, "freq_lo is NULL");
    const double lo = rebin_window(t, d->central_freq, d->dfreq, d->nout);
    if (!std::isfinite(lo)) return fail(VISTA_E_ARG, "the window's lower edge is not finite");
    *freq_lo = lo;
    return VISTA_OK;
}

int vista_rebin_rows(const vista_rebin_desc* d, int32_t n, const vista_target* t, const vista_rebin_output* o,
                     void* hip_stream, double* freq_lo, vista_timings* tim) {
    std::string why;
    if (!check_rebin_desc(d, &why)) return fail(VISTA_E_ARG, why);
    if (n < 0) return fail(VISTA_E_ARG, "n_targets must be >= 0");
    if (n > 0 && (!t || !o)) return fail(VISTA_E_ARG, "targets or outputs are NULL");
    for (int32_t i = 0; i < n; ++i) {
        const std::string at = "target " + std::to_string(i) + ": ";
        if (!check_target(nullptr, &t[i], &why)) return fail(VISTA_E_ARG, at + why);
        if (t[i].nrow == 0) continue;
        if (t[i].mem != VISTA_MEM_DEVICE) return fail(VISTA_E_ARG, at + "vista_rebin_rows needs device data");
        const vista_rebin_output& q = o[i];
        const size_t np = (size_t)t[i].npol;
        if (!q.vis) return fail(VISTA_E_ARG, at + "output vis is NULL");
        if (((uintptr_t)q.vis % (np == 1 ? 8 : 16)) || ((uintptr_t)q.flag % np) || ((uintptr_t)q.wsum % (4 * np)) ||
            ((uintptr_t)q.uvw % 8))
            return fail(VISTA_E_ARG, at + "output buffers are not aligned (vis 16 (8 for npol 1), flag npol, "
                                          "wsum 4 npol, uvw 8 bytes)");
    }
    if (n == 0) {
        if (tim) memset(tim, 0, sizeof(*tim));
        return VISTA_OK;
    }
    hipStream_t stream = (hipStream_t)hip_stream;
    return guarded(nullptr, [&]() -> int {
        Events ev;
        VISTA_HIP(hipEventRecord(ev.e[0], stream));
        DevMem mem(stream);
        // host tables: one arena, every table 256-byte aligned
        std::vector<RebinPlan> plans(n);
        std::vector<double> lo(n, 0.0);
        std::vector<size_t> off(4 * (size_t)std::max(n, 1));
        size_t bytes = 0;
        for (int32_t i = 0; i < n; ++i) {
            lo[i] = rebin_window(&t[i], d->central_freq, d->dfreq, d->nout);
            if (!std::isfinite(lo[i])) throw HipFail{hipErrorInvalidValue, "rebin window edge not finite"};
            plans[i] = plan_rebin(&t[i], lo[i], d->dfreq, d->nout);
            const RebinPlan& P = plans[i];
            off[4 * i] = bytes; bytes += align256(P.a.size() * sizeof(double));
            off[4 * i + 1] = bytes; bytes += align256(P.jstart.size() * sizeof(int32_t));
            off[4 * i + 2] = bytes; bytes += align256(std::max<size_t>(1, P.ek.size()) * sizeof(int32_t));
            off[4 * i + 3] = bytes; bytes += align256(std::max<size_t>(1, P.ef.size()) * sizeof(float));
        }
        std::vector<unsigned char> arena(std::max<size_t>(bytes, 256), 0);
        for (int32_t i = 0; i < n; ++i) {
            const RebinPlan& P = plans[i];
            memcpy(arena.data() + off[4 * i], P.a.data(), P.a.size() * sizeof(double));
            memcpy(arena.data() + off[4 * i + 1], P.jstart.data(), P.jstart.size() * sizeof(int32_t));
            if (!P.ek.empty()) memcpy(arena.data() + off[4 * i + 2], P.ek.data(), P.ek.size() * sizeof(int32_t));
            if (!P.ef.empty()) memcpy(arena.data() + off[4 * i + 3], P.ef.data(), P.ef.size() * sizeof(float));
        }
        unsigned char* darena = mem.alloc_n<unsigned char>(arena.size());
        std::vector<RebinTarget> dts(std::max(n, 1));
        for (int32_t i = 0; i < n; ++i) {
            RebinTarget& T = dts[i];
            memset(&T, 0, sizeof(T));
            T.uvw = t[i].uvw; T.vis = (const float2*)t[i].vis; T.flag = t[i].flag;
            T.out_vis = (float2*)o[i].vis; T.out_flag = o[i].flag; T.out_wsum = o[i].wsum; T.out_uvw = o[i].uvw;
            T.a = (const double*)(darena + off[4 * i]);
            T.jstart = (const int32_t*)(darena + off[4 * i + 1]);
            T.ek = (const int32_t*)(darena + off[4 * i + 2]);
            T.ef = (const float*)(darena + off[4 * i + 3]);
            T.nrow = t[i].nrow; T.nchan = t[i].nchan; T.npol = t[i].npol; T.nout = d->nout;
            T.l = plans[i].frame.l; T.m = plans[i].frame.m; T.nm1 = plans[i].nm1; T.opz = 1.0 + t[i].z;
            T.rotate = plans[i].frame.rotate;
            for (int q = 0; q < 9; ++q) T.R[q] = plans[i].frame.R[q];
        }
        // row blocks, grouped by polarisation count: a workgroup's thread groups (256 /
        // min(nout, 256) of them) take 16 rows each
        const int32_t rpb = std::min(2048, 16 * (256 / std::min(d->nout, 256)));
        std::vector<RebinBlock> blocks;
        int64_t cls[3][2] = {{0, 0}, {0, 0}, {0, 0}};   // npol 1, 2, 4: [first, count)
        const int pols[3] = {1, 2, 4};
        for (int c = 0; c < 3; ++c) {
            cls[c][0] = (int64_t)blocks.size();
            for (int32_t i = 0; i < n; ++i) {
                if (t[i].npol != pols[c]) continue;
                for (int64_t r0 = 0; r0 < t[i].nrow; r0 += rpb)
                    blocks.push_back(RebinBlock{i, (int32_t)r0, (int32_t)std::min<int64_t>(rpb, t[i].nrow - r0), 0});
            }
            cls[c][1] = (int64_t)blocks.size() - cls[c][0];
        }
        RebinTarget* dT = mem.alloc_n<RebinTarget>(dts.size());
        RebinBlock* dB = mem.alloc_n<RebinBlock>(std::max<size_t>(1, blocks.size()));
        VISTA_HIP(hipMemcpyAsync(darena, arena.data(), arena.size(), hipMemcpyHostToDevice, stream));
        VISTA_HIP(hipMemcpyAsync(dT, dts.data(), dts.size() * sizeof(RebinTarget), hipMemcpyHostToDevice, stream));
        if (!blocks.empty())
            VISTA_HIP(hipMemcpyAsync(dB, blocks.data(), blocks.size() * sizeof(RebinBlock), hipMemcpyHostToDevice,
                                     stream));
        VISTA_HIP(hipEventRecord(ev.e[1], stream));
        for (int c = 0; c < 3; ++c)
            check_launch(launch_rebin_rows(dT, dB + cls[c][0], cls[c][1], pols[c], stream), "rebin rows");
        VISTA_HIP(hipEventRecord(ev.e[2], stream));
        VISTA_HIP(hipEventRecord(ev.e[3], stream));
        VISTA_HIP(hipStreamSynchronize(stream));   // the host tables above are read until here
        mem.release();
        VISTA_HIP(hipStreamSynchronize(stream));
        if (freq_lo)
            for (int32_t i = 0; i < n; ++i) freq_lo[i] = lo[i];
        if (tim) {
            memset(tim, 0, sizeof(*tim));
            tim->bin_ms = ev.ms(0, 1);
            tim->accum_ms = ev.ms(1, 2);
            tim->total_ms = ev.ms(0, 3);
            tim->n_accum_launches = (cls[0][1] > 0) + (cls[1][1] > 0) + (cls[2][1] > 0);
        }
        return VISTA_OK;
    });
}

// -------------------------------------------------------------------- dirty image

int vista_image(const vista_grid_desc* g, const void* sum_wvis, const float* sum_w, float* image, float* beam,
                void* hip_stream, vista_timings* tim) {
    if (!g) return fail(VISTA_E_ARG, "grid descriptor is NULL");
    auto pow2 = [](int32_t n) { return n >= 2 && n <= 4096 && (n & (n - 1)) == 0; };
    if (!pow2(g->nu) || !pow2(g->nv)) return fail(VISTA_E_ARG, "vista_image needs nu and nv powers of two in 2..4096");
    if (g->nchan < 1 || g->nchan > 65535) return fail(VISTA_E_ARG, "vista_image needs nchan in 1..65535");
    if (!sum_wvis || !sum_w || !image) return fail(VISTA_E_ARG, "sum_wvis, sum_w and image are required");
    if (((uintptr_t)sum_wvis % 8) || ((uintptr_t)sum_w % 4) || ((uintptr_t)image % 4) || ((uintptr_t)beam % 4))
        return fail(VISTA_E_ARG, "arrays are not aligned to their element size");
    for (const void* ptr : {(const void*)sum_wvis, (const void*)sum_w, (const void*)image, (const void*)beam}) {
        if (!ptr) continue;
        hipPointerAttribute_t at;
        if (hipPointerGetAttributes(&at, ptr) != hipSuccess || at.type != hipMemoryTypeDevice) {
            (void)hipGetLastError();
            return fail(VISTA_E_ARG, "vista_image needs device memory");
        }
    }
    hipStream_t stream = (hipStream_t)hip_stream;
    return guarded(nullptr, [&]() -> int {
        Events ev;
        DevMem mem(stream);
        float2* tmp = (float2*)mem.alloc(image_temp_bytes(g->nu, g->nv, g->nchan));
        double* wsum = mem.alloc_n<double>(g->nchan);
        VISTA_HIP(hipEventRecord(ev.e[0], stream));
        check_launch(launch_image(sum_wvis, sum_w, image, beam, g->nu, g->nv, g->nchan, tmp,
                                  image_temp_bytes(g->nu, g->nv, g->nchan), wsum, stream),
                     "image");
        VISTA_HIP(hipEventRecord(ev.e[1], stream));
        VISTA_HIP(hipStreamSynchronize(stream));
        mem.release();
        VISTA_HIP(hipStreamSynchronize(stream));
        if (tim) {
            memset(tim, 0, sizeof(*tim));
            tim->accum_ms = ev.ms(0, 1);
            tim->total_ms = tim->accum_ms;
            tim->n_accum_launches = beam ? 5 : 3;
        }
        return VISTA_OK;
    });
}

int vista_image_noalloc(const vista_grid_desc* g, const void* sum_wvis, const float* sum_w, float* image,
                        float* beam, void* hip_stream) {
    if (!g) return fail(VISTA_E_ARG, "grid descriptor is NULL");
    auto pow2 = [](int32_t n) { return n >= 2 && n <= 4096 && (n & (n - 1)) == 0; };
    if (!pow2(g->nu) || !pow2(g->nv)) return fail(VISTA_E_ARG, "vista_image_noalloc needs nu and nv powers of two in 2..4096");
    if (g->nchan < 1 || g->nchan > 65535) return fail(VISTA_E_ARG, "vista_image_noalloc needs nchan in 1..65535");
    const size_t plane_bytes = (size_t)g->nu * g->nv * sizeof(float2);
    if (plane_bytes > kNoAllocImageStaging)
        return fail(VISTA_E_ARG, "vista_image_noalloc: one " + std::to_string(g->nu) + " x " + std::to_string(g->nv) +
                                     " plane needs " + std::to_string(plane_bytes >> 20) +
                                     " MiB of staging, more than its fixed 64 MiB scratch (nu * nv <= 8388608)");
    if (!sum_wvis || !sum_w || !image) return fail(VISTA_E_ARG, "sum_wvis, sum_w and image are required");
    if (((uintptr_t)sum_wvis % 8) || ((uintptr_t)sum_w % 4) || ((uintptr_t)image % 4) || ((uintptr_t)beam % 4))
        return fail(VISTA_E_ARG, "arrays are not aligned to their element size");
    for (const void* ptr : {(const void*)sum_wvis, (const void*)sum_w, (const void*)image, (const void*)beam}) {
        if (!ptr) continue;
        hipPointerAttribute_t at;
        if (hipPointerGetAttributes(&at, ptr) != hipSuccess || at.type != hipMemoryTypeDevice) {
            (void)hipGetLastError();
            return fail(VISTA_E_ARG, "vista_image_noalloc needs device memory");
        }
    }
    hipStream_t stream = (hipStream_t)hip_stream;
    return guarded(nullptr, [&]() -> int {
        hipError_t e = hipSuccess;
        unsigned char* base = (unsigned char*)image_noalloc_scratch(&e);
        if (!base) throw HipFail{e, "hipGetSymbolAddress(scratch)"};
        float2* tmp = (float2*)base;
        double* wsum = (double*)(base + kNoAllocImageStaging);
        check_launch(launch_image(sum_wvis, sum_w, image, beam, g->nu, g->nv, g->nchan, tmp, kNoAllocImageStaging,
                                  wsum, stream),
                     "image");
        return VISTA_OK;
    });
}

// ---------------------------------------------------------------------------- batch

int vista_batch_create(int32_t n_stacks, const vista_grid_desc* g, void* hip_stream, vista_batch** out) {
    if (!out) return fail(VISTA_E_ARG, "out is NULL");
    if (n_stacks < 1 || !g) return fail(VISTA_E_ARG, "need n_stacks >= 1 grids");
    std::string why;
    const uint32_t mode_bits = VISTA_F_KAHAN | VISTA_F_DETERMINISTIC | VISTA_F_PHASE_FP32 | VISTA_F_PLAIN_FP32;
    for (int32_t i = 0; i < n_stacks; ++i) {
        if (!check_grid(&g[i], &why)) return fail(VISTA_E_ARG, "stack " + std::to_string(i) + ": " + why);
        if ((g[i].flags & mode_bits) != (g[0].flags & mode_bits))
            return fail(VISTA_E_ARG,
                        "all stacks of a batch need the same KAHAN/DETERMINISTIC/PHASE_FP32/PLAIN_FP32 flags");
    }
    try {
        auto* b = new vista_batch();
        b->g.assign(g, g + n_stacks);
        b->stream = (hipStream_t)hip_stream;
        b->targets.resize(n_stacks);
        vista_output none{};
        none.mem = -1;
        b->reg.assign(n_stacks, none);
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
        if (h->planned && !check_plan(h->plan, &w)) return fail(VISTA_E_ARG, w);
        b->targets[stack].reserve(b->targets[stack].size() + 1);
        plan_in_background(h.get());
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

// Device bytes a streamed target occupies in staging (uvw, vis, weights, flags).
static size_t staged_bytes(const vista_target& t) {
    const size_t nr = (size_t)t.nrow, ns = nr * t.nchan * t.npol;
    const size_t b_w = (t.weight_per_chan ? ns : nr * t.npol) * sizeof(float);
    return align256(nr * 3 * sizeof(double)) + align256(ns * 8) + align256(b_w) + (t.flag ? align256(ns) : 0);
}

static int64_t default_stream_budget() {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess || fr == 0) return (int64_t)1 << 30;
    return (int64_t)(fr / 8);   // two staging buffers take a quarter of the free memory
}

int vista_batch_run(vista_batch* b) {
    if (!b) return fail(VISTA_E_ARG, "batch is NULL");
    if (b->state != 0) return fail(VISTA_E_STATE, b->state == 1 ? "batch already ran" : "batch is poisoned");
    return guarded(&b->state, [&]() -> int {
        using clk = std::chrono::steady_clock;
        const clk::time_point h0 = clk::now();
        // the batch runs on streams of its own (a capture needs a stream other than the
        // legacy default one), ordered after the caller's stream and before it again
        struct StreamGuard {
            hipStream_t s = nullptr, c = nullptr;
            std::vector<hipEvent_t> ev;
            ~StreamGuard() {
                if (c) (void)hipStreamSynchronize(c);
                if (s) (void)hipStreamSynchronize(s);
                for (auto e : ev) (void)hipEventDestroy(e);
                if (s) (void)hipStreamDestroy(s);
                if (c) (void)hipStreamDestroy(c);
            }
            hipEvent_t make(unsigned fl) {
                hipEvent_t e;
                VISTA_HIP(hipEventCreateWithFlags(&e, fl));
                ev.push_back(e);
                return e;
            }
        } g;
        VISTA_HIP(hipStreamCreateWithFlags(&g.s, hipStreamNonBlocking));
        VISTA_HIP(hipStreamCreateWithFlags(&g.c, hipStreamNonBlocking));
        hipStream_t us = b->stream;
        hipStream_t st = g.c;
        b->keep = std::make_unique<DevMem>(us, false, true);
        const size_t ns = b->g.size();
        const uint32_t flags = b->g[0].flags;
        const bool kahan = (flags & VISTA_F_KAHAN) != 0;
        b->res.assign(ns, {});
        for (size_t s = 0; s < ns; ++s) {
            const vista_grid_desc& g = b->g[s];
            const size_t nc = (size_t)g.nu * g.nv * g.nchan;
            auto& R = b->res[s];
            const vista_output& o = b->reg[s];
            if (o.mem == VISTA_MEM_DEVICE) {          // written in place
                R.vis = (float2*)o.sum_wvis; R.w = (float*)o.sum_w; R.cnt = (uint32_t*)o.count;
                R.vis64 = (double2*)o.sum_wvis64; R.w64 = (double*)o.sum_w64;
                continue;
            }
            const bool any = o.mem < 0;               // nothing registered: keep everything
            if (any || o.sum_wvis) R.vis = b->keep->alloc_n<float2>(nc);
            if (any || o.sum_w) R.w = b->keep->alloc_n<float>(nc);
            if (any || o.count) R.cnt = b->keep->alloc_n<uint32_t>(nc);
            if (any || o.sum_wvis64) R.vis64 = b->keep->alloc_n<double2>(nc);
            if (any || o.sum_w64) R.w64 = b->keep->alloc_n<double>(nc);
        }
        // ---- waves: device-resident targets go in the first; targets in host memory are
        // packed, in order, into waves of at most `budget` staged bytes
        const int64_t budget = b->stream_budget > 0 ? b->stream_budget : default_stream_budget();
        struct Item { int32_t stack; HostTarget* h; size_t off; };
        std::vector<std::vector<Item>> waves(1);
        std::vector<size_t> wbytes(1, 0);
        for (size_t s = 0; s < ns; ++s)
            for (auto& hp : b->targets[s]) {
                HostTarget* h = hp.get();
                if (h->t.nrow == 0 || h->t.mem == VISTA_MEM_DEVICE) {
                    waves[0].push_back({(int32_t)s, h, 0});
                    continue;
                }
                const size_t nb = staged_bytes(h->t);
                if ((int64_t)nb > budget) throw NoMem{"a target is larger than the stream budget"};
                if (wbytes.back() > 0 && (int64_t)(wbytes.back() + nb) > budget) {
                    waves.emplace_back();
                    wbytes.push_back(0);
                }
                waves.back().push_back({(int32_t)s, h, wbytes.back()});
                wbytes.back() += nb;
            }
        const size_t nw = waves.size();
        vlog(2, "batch plan: %zu stack(s), %zu wave(s), stream budget %lld bytes", ns, nw, (long long)budget);
        // a stack takes part in the waves holding its targets (a stack without targets in
        // the first, so that its cells are written)
        std::vector<std::vector<char>> member(nw, std::vector<char>(ns, 0));
        for (size_t w = 0; w < nw; ++w)
            for (auto& it : waves[w]) member[w][it.stack] = 1;
        for (size_t s = 0; s < ns; ++s)
            if (b->targets[s].empty()) member[0][s] = 1;
        std::vector<int> last(ns, -1), nwaves(ns, 0);
        for (size_t w = 0; w < nw; ++w)
            for (size_t s = 0; s < ns; ++s)
                if (member[w][s]) {
                    last[s] = (int)w;
                    ++nwaves[s];
                }
        // ---- carried state of the stacks spread over several waves
        std::vector<float*> cs_s(ns, nullptr), cs_c(ns, nullptr);
        std::vector<uint32_t*> cs_n(ns, nullptr);
        for (size_t s = 0; s < ns; ++s) {
            if (nwaves[s] < 2) continue;
            const int64_t nc = carried_state_cells(b->g[s], b->tune);
            cs_s[s] = b->keep->alloc_n<float>(3 * nc);
            cs_n[s] = b->keep->alloc_n<uint32_t>(nc);
            if (kahan) cs_c[s] = b->keep->alloc_n<float>(3 * nc);
        }
        unsigned long long* d_stats = b->keep->alloc_n<unsigned long long>(8 * ns);
        size_t maxw = 0;
        for (size_t w = 0; w < nw; ++w) maxw = std::max(maxw, wbytes[w]);
        unsigned char* stage[2] = {nullptr, nullptr};
        if (maxw > 0) {
            stage[0] = b->keep->alloc_n<unsigned char>(maxw);
            if (nw > 1) stage[1] = b->keep->alloc_n<unsigned char>(maxw);
        }
        const clk::time_point h1 = clk::now();
        // ---- the batch's streams start after the caller's stream (and these allocations)
        hipEvent_t e_in = g.make(hipEventDisableTiming);
        VISTA_HIP(hipEventRecord(e_in, us));
        VISTA_HIP(hipStreamWaitEvent(st, e_in, 0));
        VISTA_HIP(hipStreamWaitEvent(g.s, e_in, 0));
        for (size_t s = 0; s < ns; ++s) {
            if (!cs_s[s]) continue;
            const int64_t nc = carried_state_cells(b->g[s], b->tune);
            check_launch(launch_fill_u32((uint32_t*)cs_s[s], 0u, 3 * nc, st), "fill");
            check_launch(launch_fill_u32(cs_n[s], 0u, nc, st), "fill");
            if (cs_c[s]) check_launch(launch_fill_u32((uint32_t*)cs_c[s], 0u, 3 * nc, st), "fill");
        }
        check_launch(launch_fill_u64(d_stats, 0ull, 8 * (int64_t)ns, st), "fill");
        // ---- one host launch per wave
        Launcher ln(st, b->tune, flags);
        std::vector<std::vector<StackJob>> wj(nw);
        std::vector<HostLaunch> hl(nw);
        Capacity cap;
        for (size_t w = 0; w < nw; ++w) {
            std::vector<int> slot(ns, -1);
            for (size_t s = 0; s < ns; ++s) {
                if (!member[w][s]) continue;
                StackJob J;
                J.g = &b->g[s];
                J.index = (int32_t)s;
                auto& R = b->res[s];
                J.out.sum_wvis = R.vis; J.out.sum_w = R.w; J.out.count = R.cnt;
                J.out.sum_wvis64 = R.vis64; J.out.sum_w64 = R.w64;
                J.out.mem = VISTA_MEM_DEVICE;
                J.carry = nwaves[s] > 1 ? 1 : 0;
                J.last = (int)w == last[s] ? 1 : 0;
                J.st_s = cs_s[s]; J.st_c = cs_c[s]; J.st_n = cs_n[s];
                slot[s] = (int)wj[w].size();
                wj[w].push_back(J);
            }
            for (auto& it : waves[w]) wj[w][slot[it.stack]].targets.push_back(it.h);
            hl[w] = build_launch(wj[w], b->tune, ln.jsub());
            cap = cap.max_with(Capacity::of(hl[w]));
        }
        ln.reserve(cap);
        std::vector<hipEvent_t> copied(nw), done(nw), t0(nw), t1(nw), t2(nw), c0(nw), c1(nw);
        for (size_t w = 0; w < nw; ++w) {
            copied[w] = g.make(hipEventDisableTiming);
            done[w] = g.make(hipEventDisableTiming);
            t0[w] = g.make(hipEventDefault); t1[w] = g.make(hipEventDefault); t2[w] = g.make(hipEventDefault);
            c0[w] = g.make(hipEventDefault); c1[w] = g.make(hipEventDefault);
        }
        hipEvent_t e_start = g.make(hipEventDefault), e_end = g.make(hipEventDefault);
        const clk::time_point h2 = clk::now();
        VISTA_HIP(hipEventRecord(e_start, st));
        // device pointers of wave w's targets; streamed ones are copied into its buffer
        auto stage_wave = [&](size_t w) {
            HostLaunch& h = hl[w];
            unsigned char* base = stage[w & 1];
            if (w >= 2) VISTA_HIP(hipStreamWaitEvent(g.s, done[w - 2], 0));   // that buffer's last reader
            VISTA_HIP(hipEventRecord(c0[w], g.s));
            for (size_t i = 0; i < h.dts.size(); ++i) {
                DevTarget& T = h.dts[i];
                const vista_target& t = h.hts[i]->t;
                if (t.mem == VISTA_MEM_DEVICE) {
                    T.uvw = t.uvw; T.vis = (const float2*)t.vis; T.weight = t.weight; T.flag = t.flag;
                    continue;
                }
                size_t off = 0;
                for (auto& it : waves[w])
                    if (it.h == h.hts[i]) off = it.off;
                const size_t nr = (size_t)t.nrow, nsm = nr * t.nchan * t.npol;
                const size_t b_w = (t.weight_per_chan ? nsm : nr * t.npol) * sizeof(float);
                unsigned char* p = base + off;
                VISTA_HIP(hipMemcpyAsync(p, t.uvw, nr * 24, hipMemcpyHostToDevice, g.s));
                T.uvw = (const double*)p; p += align256(nr * 24);
                VISTA_HIP(hipMemcpyAsync(p, t.vis, nsm * 8, hipMemcpyHostToDevice, g.s));
                T.vis = (const float2*)p; p += align256(nsm * 8);
                VISTA_HIP(hipMemcpyAsync(p, t.weight, b_w, hipMemcpyHostToDevice, g.s));
                T.weight = (const float*)p; p += align256(b_w);
                T.flag = nullptr;
                if (t.flag) {
                    VISTA_HIP(hipMemcpyAsync(p, t.flag, nsm, hipMemcpyHostToDevice, g.s));
                    T.flag = (const uint8_t*)p;
                }
            }
            VISTA_HIP(hipEventRecord(c1[w], g.s));
            VISTA_HIP(hipEventRecord(copied[w], g.s));
        };
        int64_t nrec_total = 0;
        stage_wave(0);
        for (size_t w = 0; w < nw; ++w) {
            if (w + 1 < nw) stage_wave(w + 1);     // overlaps this wave's compute
            VISTA_HIP(hipStreamWaitEvent(st, copied[w], 0));
            VISTA_HIP(hipEventRecord(t0[w], st));
            const int64_t nrec = ln.prepare(hl[w], d_stats);
            nrec_total += nrec;
            Capacity c = ln.capacity();
            c.recs = nrec;
            ln.reserve(c);
            ln.replay(t1[w]);
            VISTA_HIP(hipEventRecord(t2[w], st));
            VISTA_HIP(hipEventRecord(done[w], st));
        }
        std::vector<unsigned long long> stv(8 * ns);
        VISTA_HIP(hipMemcpyAsync(stv.data(), d_stats, stv.size() * 8, hipMemcpyDeviceToHost, st));
        VISTA_HIP(hipEventRecord(e_end, st));
        VISTA_HIP(hipStreamWaitEvent(us, e_end, 0));   // the caller's stream resumes after the batch
        VISTA_HIP(hipStreamSynchronize(st));
        VISTA_HIP(hipStreamSynchronize(g.s));
        // per-stack classification over all waves
        std::vector<StackJob> all(ns);
        for (size_t s = 0; s < ns; ++s) {
            all[s].g = &b->g[s];
            all[s].index = (int32_t)s;
            for (auto& hp : b->targets[s]) all[s].targets.push_back(hp.get());
        }
        collect_stats(all, stv);
        for (size_t s = 0; s < ns; ++s) {
            b->res[s].st = all[s].stats;
            b->res[s].overflow = all[s].overflow;
        }
        vista_timings& T = b->tim;
        memset(&T, 0, sizeof(T));
        auto ms = [](hipEvent_t a, hipEvent_t z) {
            float t = 0;
            (void)hipEventElapsedTime(&t, a, z);
            return (double)t;
        };
        for (size_t w = 0; w < nw; ++w) {
            T.bin_ms += ms(t0[w], t1[w]);
            T.accum_ms += ms(t1[w], t2[w]);
            if (wbytes[w] > 0) T.h2d_ms += ms(c0[w], c1[w]);
        }
        T.total_ms = ms(e_start, e_end);
        T.n_records = nrec_total;
        T.n_units = cap.units;
        T.n_accum_launches = (int32_t)nw;
        T.n_waves = (int32_t)nw;
        auto host_ms = [](clk::time_point a, clk::time_point z) {
            return std::chrono::duration<double, std::milli>(z - a).count();
        };
        vlog(1, "batch run: %zu stack(s), %zu wave(s), %lld records; binning %.3f ms, accumulation %.3f ms, "
                "input copies %.3f ms, total %.3f ms; host set-up before the first launch %.1f ms "
                "(allocation %.1f ms, launch build %.1f ms)",
             ns, nw, (long long)nrec_total, T.bin_ms, T.accum_ms, T.h2d_ms, T.total_ms, host_ms(h0, h2),
             host_ms(h0, h1), host_ms(h1, h2));
        b->state = 1;
        return VISTA_OK;
    });
}

int vista_batch_set_output(vista_batch* b, int32_t stack, const vista_output* o) {
    if (!b || !o) return fail(VISTA_E_ARG, "NULL argument");
    if (b->state != 0) return fail(VISTA_E_STATE, "batch already ran");
    if (stack < 0 || stack >= (int32_t)b->g.size()) return fail(VISTA_E_ARG, "stack index out of range");
    std::string why;
    if (!check_output(o, &why)) return fail(VISTA_E_ARG, why);
    b->reg[stack] = *o;
    return VISTA_OK;
}

int vista_batch_finalize(vista_batch* b, int32_t stack, const vista_output* o, vista_stats* st) {
    if (!b) return fail(VISTA_E_ARG, "batch is NULL");
    if (b->state != 1) return fail(VISTA_E_STATE, b->state == 0 ? "batch has not run" : "batch is poisoned");
    if (stack < 0 || stack >= (int32_t)b->g.size()) return fail(VISTA_E_ARG, "stack index out of range");
    std::string why;
    if (!check_output(o, &why)) return fail(VISTA_E_ARG, why);
    const vista_output& reg = b->reg[stack];
    if (!o && reg.mem >= 0 && reg.mem != VISTA_MEM_DEVICE) o = &reg;   // registered host outputs
    return guarded(&b->state, [&]() -> int {
        const vista_grid_desc& g = b->g[stack];
        size_t nc = (size_t)g.nu * g.nv * g.nchan;
        auto& R = b->res[stack];
        if (o) {
            hipMemcpyKind kind = o->mem == VISTA_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
            auto copy = [&](void* dst, const void* src, size_t n, const char* what) {
                if (!dst || dst == src) return;
                if (!src) throw HipFail{hipErrorInvalidValue, std::string("output not kept by the run: ") + what};
                VISTA_HIP(hipMemcpyAsync(dst, src, n, kind, b->stream));
            };
            copy(o->sum_wvis, R.vis, nc * 8, "sum_wvis");
            copy(o->sum_w, R.w, nc * 4, "sum_w");
            copy(o->count, R.cnt, nc * 4, "count");
            copy(o->sum_wvis64, R.vis64, nc * 16, "sum_wvis64");
            copy(o->sum_w64, R.w64, nc * 8, "sum_w64");
        }
        VISTA_HIP(hipStreamSynchronize(b->stream));
        if (st) *st = R.st;
        if (R.overflow) return fault_fail(R.overflow);
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
    if (s->state != 0) return fail(VISTA_E_STATE, "stack is not open");
    for (auto& h : s->targets)
        if (h->t.mem != VISTA_MEM_DEVICE && h->t.nrow > 0)
            return fail(VISTA_E_ARG, "autotuning needs VISTA_MEM_DEVICE targets");
    return guarded(nullptr, [&]() -> int {
        DevMem mem(s->stream);
        std::vector<StackJob> jobs(1);
        jobs[0].g = &s->g;
        for (auto& h : s->targets) jobs[0].targets.push_back(h.get());
        bool cached = false;
        const Tuning t = autotune_cached(jobs, s->g.flags, s->stream, &cached, [&] { scratch_outputs(jobs[0], mem); });
        mem.release();
        VISTA_HIP(hipStreamSynchronize(s->stream));
        s->tune = t;
        s->tune_set = true;
        to_public(t, best);
        return VISTA_OK;
    });
}

int vista_batch_autotune(vista_batch* b, vista_tuning* best) {
    if (!b) return fail(VISTA_E_ARG, "batch is NULL");
    if (b->state != 0) return fail(VISTA_E_STATE, "batch already ran");
    for (auto& ts : b->targets)
        for (auto& h : ts)
            if (h->t.mem != VISTA_MEM_DEVICE && h->t.nrow > 0)
                return fail(VISTA_E_ARG, "autotuning needs VISTA_MEM_DEVICE targets");
    return guarded(nullptr, [&]() -> int {
        DevMem mem(b->stream);
        std::vector<StackJob> jobs(b->g.size());
        for (size_t s = 0; s < jobs.size(); ++s) {
            jobs[s].g = &b->g[s];
            for (auto& h : b->targets[s]) jobs[s].targets.push_back(h.get());
        }
        bool cached = false;
        const Tuning t = autotune_cached(jobs, b->g[0].flags, b->stream, &cached, [&] {
            for (auto& J : jobs) scratch_outputs(J, mem);
        });
        mem.release();
        VISTA_HIP(hipStreamSynchronize(b->stream));
        b->tune = t;
        b->tune_set = true;
        to_public(t, best);
        return VISTA_OK;
    });
}

}  // extern "C"
