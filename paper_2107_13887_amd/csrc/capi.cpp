// C entry points: context and pool, argument validation, dispatch to the kernels.
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "basis.h"
#include "internal.h"

namespace rbf {

// hipcc gives every translation unit with kernels a constructor that registers its GPU code
// object and hands the matching unregistration to atexit(); exit() runs such handlers in reverse
// order of registration. Initialising the HIP runtime first (priority 101 sorts this constructor
// ahead of those at the default priority) makes every exit handler the runtime, or a profiler
// attached to it, registers while it initialises older than the unregistrations, so those run
// first, against a runtime that is still whole. Without a device the call just fails.
__attribute__((constructor(101))) static void init_runtime_before_modules() { (void)hipInit(0); }

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

rbf_status fail(rbf_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

double now_seconds()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---- pool --------------------------------------------------------------------------------------
size_t Pool::round_up(size_t b)
{
    if (b < 512) return 512;
    if (b <= (size_t(1) << 26)) {  // power-of-two classes up to 64 MiB
        size_t c = 512;
        while (c < b) c <<= 1;
        return c;
    }
    const size_t g = size_t(2) << 20;  // 2 MiB granules above
    return (b + g - 1) / g * g;
}

void Pool::reclaim_locked()
{
    for (auto it = deferred_.begin(); it != deferred_.end();) {
        if (hipEventQuery(it->ev) == hipSuccess) {
            (void)hipEventDestroy(it->ev);
            size_t sz = size_of_[it->p];
            free_.emplace(sz, it->p);
            live_ -= sz;
            it = deferred_.erase(it);
        } else {
            ++it;
        }
    }
}

rbf_status Pool::alloc(void **p, size_t bytes)
{
    std::lock_guard<std::mutex> lk(mu_);
    reclaim_locked();
    const size_t need = round_up(bytes ? bytes : 1);
    auto it = free_.lower_bound(need);
    if (it != free_.end() && it->first <= need + need / 2 + 4096) {
        *p = it->second;
        live_ += it->first;
        free_.erase(it);
        return RBF_OK;
    }
    auto release_cached = [&]() {
        for (auto &kv : free_) {
            (void)hipFree(kv.second);
            held_ -= kv.first;
            size_of_.erase(kv.second);
        }
        free_.clear();
    };
    if (held_ + need > budget_) {
        release_cached();
        if (held_ + need > budget_ && !deferred_.empty()) {
            for (auto &d : deferred_) (void)hipEventSynchronize(d.ev);
            reclaim_locked();
            release_cached();
        }
        if (held_ + need > budget_)
            return fail(RBF_E_NOMEM, "HBM budget exceeded: %llu held + %llu requested > %llu budget",
                        (unsigned long long)held_, (unsigned long long)need,
                        (unsigned long long)budget_);
    }
    (void)hipSetDevice(device_);
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, need);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release_cached();
        e = hipMalloc(&q, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(RBF_E_NOMEM, "hipMalloc(%llu) failed: %s", (unsigned long long)need,
                        hipGetErrorString(e));
        }
    }
    held_ += need;
    live_ += need;
    size_of_[q] = need;
    *p = q;
    return RBF_OK;
}

void Pool::free_now(void *p)
{
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = size_of_.find(p);
    if (it == size_of_.end()) return;
    free_.emplace(it->second, p);
    live_ -= it->second;
}

rbf_status Pool::free_after(void *p, hipStream_t s)
{
    if (!p) return RBF_OK;
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(ev, s) != hipSuccess) {
        // Fall back to waiting for the stream: correctness over reuse.
        (void)hipStreamSynchronize(s);
        free_now(p);
        return RBF_OK;
    }
    std::lock_guard<std::mutex> lk(mu_);
    deferred_.push_back(Deferred{p, ev});
    return RBF_OK;
}

Pool::~Pool()
{
    std::lock_guard<std::mutex> lk(mu_);
    for (auto &d : deferred_) {
        (void)hipEventSynchronize(d.ev);
        (void)hipEventDestroy(d.ev);
    }
    deferred_.clear();
    for (auto &kv : size_of_) (void)hipFree(kv.first);
    size_of_.clear();
    free_.clear();
}

// ---- kernel timers ----------------------------------------------------------------------------
hipEvent_t KernelTimers::take()
{
    std::lock_guard<std::mutex> lk(mu);
    if (!spare.empty()) {
        hipEvent_t e = spare.back();
        spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void KernelTimers::begin(hipEvent_t *a, hipStream_t s)
{
    *a = nullptr;
    if (!enabled) return;
    *a = take();
    if (*a && hipEventRecord(*a, s) != hipSuccess) *a = nullptr;
}

void KernelTimers::end(const char *name, hipEvent_t a, hipStream_t s)
{
    if (!enabled || !a) return;
    hipEvent_t b = take();
    if (!b) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(mu);
    pending.push_back(Pending{name, a, b});
}

void KernelTimers::pair(hipEvent_t *a, hipEvent_t *b)
{
    *a = *b = nullptr;
    if (!enabled) return;
    *a = take();
    *b = take();
    if (!*a || !*b) {
        std::lock_guard<std::mutex> lk(mu);
        if (*a) spare.push_back(*a);
        if (*b) spare.push_back(*b);
        *a = *b = nullptr;
    }
}

void KernelTimers::add(const char *name, hipEvent_t a, hipEvent_t b)
{
    if (!a || !b) return;
    std::lock_guard<std::mutex> lk(mu);
    pending.push_back(Pending{name, a, b});
}

unsigned long long *KernelTimers::counter(const char *name)
{
    std::lock_guard<std::mutex> lk(mu);
    if (!count_pairs || !dev_count) return nullptr;
    auto it = slot.find(name);
    if (it == slot.end()) {
        if ((int)slot.size() >= N_COUNT) return nullptr;
        it = slot.emplace(name, (int)slot.size()).first;
    }
    return dev_count + it->second;
}

KernelTimers::~KernelTimers()
{
    for (auto &p : pending) {
        (void)hipEventSynchronize(p.b);
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : spare) (void)hipEventDestroy(e);
    if (dev_count) (void)hipFree(dev_count);
}

void KernelTimers::resolve()
{
    std::lock_guard<std::mutex> lk(mu);
    for (auto &p : pending) {
        float ms = 0.0f;
        (void)hipEventSynchronize(p.b);
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto &t = total[p.name];
            t.first += ms;
            t.second += 1;
        }
        spare.push_back(p.a);
        spare.push_back(p.b);
    }
    pending.clear();
}

// ---- validation -------------------------------------------------------------------------------
rbf_status check_precision(int32_t precision, const int32_t *level_precision, int32_t n_levels)
{
    if (precision != RBF_FP64 && precision != RBF_MIXED) return fail(RBF_E_INVALID, "bad precision %d", precision);
    if (level_precision)
        for (int l = 0; l < n_levels; ++l)
            if (level_precision[l] != RBF_FP64 && level_precision[l] != RBF_MIXED)
                return fail(RBF_E_INVALID, "bad level_precision[%d] = %d", l, level_precision[l]);
    return RBF_OK;
}

// Device address of the fixed scratch array, looked up once per device (with that device
// current) and kept for the process: each device holds its own copy of the array.
static rbf_status scratch_for_device(int device, void **ptr)
{
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;                    // trivially destructible, as is the table
    static void *addr[MAX_DEVICES] = {};
    if (device < 0 || device >= MAX_DEVICES) return fail(RBF_E_INVALID, "device %d out of range", device);
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) RBF_TRY(noalloc_scratch_address(&addr[device]));
    *ptr = addr[device];
    return RBF_OK;
}

rbf_status validate_params(const rbf_greedy_params &p, int64_t n_s)
{
    if (p.dim != 2 && p.dim != 3) return fail(RBF_E_INVALID, "dim must be 2 or 3 (got %d)", p.dim);
    if (p.n_levels < 1 || p.n_levels > RBF_MAX_LEVELS)
        return fail(RBF_E_INVALID, "n_levels must be in 1..%d (got %d)", RBF_MAX_LEVELS, p.n_levels);
    if (n_s < 1 || n_s > (int64_t(1) << 31) - 1) return fail(RBF_E_INVALID, "n_s out of range");
    for (int l = 0; l < p.n_levels; ++l)
        if (!(p.radius[l] > 0.0) || !std::isfinite(p.radius[l]))
            return fail(RBF_E_INVALID, "radius[%d] must be finite and > 0", l);
    if (!(p.eps_abs >= 0.0) || !std::isfinite(p.eps_abs))
        return fail(RBF_E_INVALID, "eps_abs must be finite and >= 0");
    if (!(p.level_reduction > 0.0 && p.level_reduction <= 1.0))
        return fail(RBF_E_INVALID, "level_reduction must be in (0, 1]");
    if (p.max_ctrl_total < 1) return fail(RBF_E_INVALID, "max_ctrl_total must be >= 1");
    if (p.precision != RBF_FP64 && p.precision != RBF_MIXED)
        return fail(RBF_E_INVALID, "unknown precision %d", p.precision);
    if (!basis_valid(p.basis)) return fail(RBF_E_INVALID, "unknown basis %d", p.basis);
    if (p.seed_off) {
        if (p.seed_off[0] != 0) return fail(RBF_E_INVALID, "seed_off[0] must be 0");
        for (int l = 0; l < p.n_levels; ++l) {
            if (p.seed_off[l + 1] < p.seed_off[l]) return fail(RBF_E_INVALID, "seed_off not monotone");
            std::vector<int64_t> seen;
            for (int32_t k = p.seed_off[l]; k < p.seed_off[l + 1]; ++k) {
                int64_t q = p.seed_idx ? p.seed_idx[k] : -1;
                if (q < 0 || q >= n_s) return fail(RBF_E_INVALID, "seed index %lld out of range", (long long)q);
                for (int64_t s : seen)
                    if (s == q) return fail(RBF_E_INVALID, "seed %lld repeated in level %d", (long long)q, l);
                seen.push_back(q);
            }
        }
    }
    return RBF_OK;
}

}  // namespace rbf

using namespace rbf;

extern "C" {

const char *rbf_status_str(rbf_status s)
{
    switch (s) {
    case RBF_OK: return "ok";
    case RBF_W_CAP: return "warning: control-point cap reached";
    case RBF_W_BREAKDOWN: return "warning: Cholesky breakdown stopped a level";
    case RBF_E_INVALID: return "invalid argument";
    case RBF_E_NOMEM: return "out of memory (HBM budget)";
    case RBF_E_NOT_SPD: return "matrix not positive definite";
    case RBF_E_DEVICE: return "device error";
    case RBF_E_NOT_FOUND: return "not found";
    case RBF_E_BUSY: return "busy";
    default: return "unknown status";
    }
}

const char *rbf_last_error(void) { return g_err; }

double rbf_now(void) { return now_seconds(); }

rbf_status rbf_ctx_create(int32_t device, uint64_t budget, rbf_ctx *out)
{
    if (!out) return fail(RBF_E_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    RBF_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        return fail(RBF_E_INVALID, "device %d out of range (%d devices)", device, count);
    RBF_HIP(hipSetDevice(device));
    auto ctx = std::make_unique<rbf_ctx_s>();
    ctx->device = device;
    RBF_HIP(hipGetDeviceProperties(&ctx->prop, device));
    ctx->n_cu = ctx->prop.multiProcessorCount > 0 ? ctx->prop.multiProcessorCount : 256;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        RBF_HIP(hipMemGetInfo(&fr, &tot));
        budget = (uint64_t)(0.9 * (double)fr);
    }
    ctx->pool = std::make_unique<Pool>(device, budget);
    RBF_TRY(scratch_for_device(device, &ctx->noalloc_scratch));
    *out = ctx.release();
    return RBF_OK;
}

rbf_status rbf_ctx_destroy(rbf_ctx ctx)
{
    if (!ctx) return fail(RBF_E_INVALID, "ctx is NULL");
    (void)hipSetDevice(ctx->device);
    server_shutdown(ctx);
    {
        std::lock_guard<std::mutex> lk(ctx->geom_mu);
        ctx->geoms.clear();
    }
    (void)hipDeviceSynchronize();
    ctx->pool.reset();
    delete ctx;
    return RBF_OK;
}

uint64_t rbf_ctx_bytes_in_use(rbf_ctx ctx) { return ctx && ctx->pool ? ctx->pool->in_use() : 0; }

rbf_status rbf_ctx_set_timing(rbf_ctx ctx, int32_t enabled)
{
    if (!ctx) return fail(RBF_E_INVALID, "ctx is NULL");
    ctx->timers.resolve();
    RBF_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(ctx->timers.mu);
    ctx->timers.enabled = (enabled & 1) != 0;
    ctx->timers.count_pairs = (enabled & 2) != 0;
    ctx->timers.total.clear();
    if (ctx->timers.count_pairs && !ctx->timers.dev_count)
        RBF_HIP(hipMalloc((void **)&ctx->timers.dev_count, sizeof(unsigned long long) * KernelTimers::N_COUNT));
    if (ctx->timers.dev_count) {
        RBF_HIP(hipDeviceSynchronize());
        RBF_HIP(hipMemset(ctx->timers.dev_count, 0, sizeof(unsigned long long) * KernelTimers::N_COUNT));
    }
    return RBF_OK;
}

rbf_status rbf_ctx_kernel_pairs(rbf_ctx ctx, const char *kernel, int64_t *pairs)
{
    if (!ctx || !kernel || !pairs) return fail(RBF_E_INVALID, "NULL argument");
    ctx->timers.resolve();
    RBF_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(ctx->timers.mu);
    *pairs = 0;
    auto it = ctx->timers.slot.find(kernel);
    if (it == ctx->timers.slot.end() || !ctx->timers.dev_count) return RBF_OK;
    RBF_HIP(hipDeviceSynchronize());
    unsigned long long v = 0;
    RBF_HIP(hipMemcpy(&v, ctx->timers.dev_count + it->second, sizeof v, hipMemcpyDeviceToHost));
    *pairs = (int64_t)v;
    return RBF_OK;
}

rbf_status rbf_ctx_kernel_time(rbf_ctx ctx, const char *kernel, double *total_ms, int64_t *launches)
{
    if (!ctx || !kernel || !total_ms || !launches) return fail(RBF_E_INVALID, "NULL argument");
    ctx->timers.resolve();
    std::lock_guard<std::mutex> lk(ctx->timers.mu);
    auto it = ctx->timers.total.find(kernel);
    *total_ms = it == ctx->timers.total.end() ? 0.0 : it->second.first;
    *launches = it == ctx->timers.total.end() ? 0 : it->second.second;
    return RBF_OK;
}

rbf_status rbf_greedy_select(rbf_ctx ctx, const rbf_greedy_params *params, int64_t n_s,
                             const double *xs, const double *ds, rbf_ctrl_set *out, void *stream)
{
    if (!ctx || !params || !out) return fail(RBF_E_INVALID, "NULL context, params or out");
    RBF_TRY(validate_params(*params, n_s));
    if (!xs || !ds || !out->ctrl_idx || !out->xc || !out->alpha)
        return fail(RBF_E_INVALID, "NULL device array");
    if (out->capacity < params->max_ctrl_total)
        return fail(RBF_E_INVALID, "out->capacity %lld < max_ctrl_total %lld",
                    (long long)out->capacity, (long long)params->max_ctrl_total);
    RBF_HIP(hipSetDevice(ctx->device));
    return run_greedy(ctx, *params, n_s, xs, ds, out, (hipStream_t)stream);
}

rbf_status rbf_solve_weights(rbf_ctx ctx, int32_t dim, double radius, int64_t n_c, const double *xc,
                             const double *dsc, double *alpha, int32_t basis, void *stream)
{
    if (!ctx) return fail(RBF_E_INVALID, "ctx is NULL");
    if (dim != 2 && dim != 3) return fail(RBF_E_INVALID, "dim must be 2 or 3");
    if (!(radius > 0.0) || !std::isfinite(radius)) return fail(RBF_E_INVALID, "radius must be > 0");
    if (n_c < 1 || n_c > 65536) return fail(RBF_E_INVALID, "n_c must be in 1..65536");
    if (!xc || !dsc || !alpha) return fail(RBF_E_INVALID, "NULL device array");
    RBF_HIP(hipSetDevice(ctx->device));
    if (!basis_valid(basis)) return fail(RBF_E_INVALID, "unknown basis %d", basis);
    return run_solve_weights(ctx, dim, radius, n_c, xc, dsc, alpha, basis, (hipStream_t)stream);
}

static rbf_status check_levels(int32_t n_levels, const double *radius, const double *D,
                               const int32_t *level_off, int64_t ld_ctrl)
{
    if (n_levels < 1 || n_levels > RBF_MAX_LEVELS) return fail(RBF_E_INVALID, "n_levels out of range");
    if (!radius || !level_off) return fail(RBF_E_INVALID, "NULL radius or level_off");
    if (level_off[0] < 0) return fail(RBF_E_INVALID, "level_off[0] < 0");
    for (int l = 0; l < n_levels; ++l) {
        if (!(radius[l] > 0.0) || !std::isfinite(radius[l]))
            return fail(RBF_E_INVALID, "radius[%d] must be finite and > 0", l);
        if (D && (!(D[l] > 0.0) || !std::isfinite(D[l])))
            return fail(RBF_E_INVALID, "D[%d] must be finite and > 0", l);
        if (level_off[l + 1] < level_off[l]) return fail(RBF_E_INVALID, "level_off not monotone");
    }
    if (level_off[n_levels] > ld_ctrl) return fail(RBF_E_INVALID, "level_off exceeds ld_ctrl");
    return RBF_OK;
}

// Validated problem of a plain volume update (shared by the pool and the allocation-free forms).
static rbf_status volume_problem(rbf_ctx ctx, int32_t dim, int32_t n_levels, const double *radius,
                                 const double *D, const int32_t *level_off, int64_t ld_ctrl,
                                 const double *xc, const double *alpha, int64_t n_v, const double *xv,
                                 const double *dwall, double *dv, int32_t precision,
                                 const int32_t *level_precision, int32_t basis, SumProblem &pb)
{
    if (!ctx) return fail(RBF_E_INVALID, "ctx is NULL");
    if (dim != 2 && dim != 3) return fail(RBF_E_INVALID, "dim must be 2 or 3");
    if (!D) return fail(RBF_E_INVALID, "D is NULL");
    RBF_TRY(check_levels(n_levels, radius, D, level_off, ld_ctrl));
    if (n_v < 0 || n_v > (int64_t(1) << 31) - 1) return fail(RBF_E_INVALID, "n_v out of range");
    RBF_TRY(check_precision(precision, level_precision, n_levels));
    if (!basis_valid(basis)) return fail(RBF_E_INVALID, "unknown basis %d", basis);
    if (n_v > 0 && (!xv || !dwall || !dv || (level_off[n_levels] > level_off[0] && (!xc || !alpha))))
        return fail(RBF_E_INVALID, "NULL device array");
    pb.dim = dim;
    pb.n_levels = n_levels;
    for (int l = 0; l < n_levels; ++l)
        pb.lv[l] = SumLevel{1.0 / radius[l], D[l], level_off[l], level_off[l + 1],
                            (level_precision ? level_precision[l] : precision) == RBF_MIXED};
    pb.ld_ctrl = ld_ctrl;
    pb.xc = xc;
    pb.alpha = alpha;
    pb.n_p = n_v;
    pb.xp = xv;
    pb.dwall = dwall;
    pb.out = dv;
    pb.sign = -1.0;
    pb.precision = precision;
    pb.basis = basis;
    return RBF_OK;
}

rbf_status rbf_volume_update(rbf_ctx ctx, int32_t dim, int32_t n_levels, const double *radius,
                             const double *D, const int32_t *level_off, int64_t ld_ctrl,
                             const double *xc, const double *alpha, int64_t n_v, const double *xv,
                             const double *dwall, double *dv, int32_t precision,
                             const int32_t *level_precision, int32_t basis, void *stream)
{
    SumProblem pb;
    RBF_TRY(volume_problem(ctx, dim, n_levels, radius, D, level_off, ld_ctrl, xc, alpha, n_v, xv, dwall, dv,
                           precision, level_precision, basis, pb));
    if (n_v == 0) return RBF_OK;
    RBF_HIP(hipSetDevice(ctx->device));
    return run_kernel_sum(ctx, pb, (hipStream_t)stream);
}

rbf_status rbf_volume_update_noalloc(rbf_ctx ctx, int32_t dim, int32_t n_levels, const double *radius,
                                     const double *D, const int32_t *level_off, int64_t ld_ctrl,
                                     const double *xc, const double *alpha, int64_t n_v, const double *xv,
                                     const double *dwall, double *dv, int32_t precision,
                                     const int32_t *level_precision, int32_t basis, void *stream)
{
    SumProblem pb;
    RBF_TRY(volume_problem(ctx, dim, n_levels, radius, D, level_off, ld_ctrl, xc, alpha, n_v, xv, dwall, dv,
                           precision, level_precision, basis, pb));
    if (n_v > RBF_NOALLOC_MAX_POINTS)
        return fail(RBF_E_INVALID, "n_v = %lld exceeds RBF_NOALLOC_MAX_POINTS (%d) of the allocation-free call",
                    (long long)n_v, RBF_NOALLOC_MAX_POINTS);
    if (!ctx->noalloc_scratch) return fail(RBF_E_DEVICE, "no fixed scratch on device %d", ctx->device);
    if (n_v == 0) return RBF_OK;
    RBF_HIP(hipSetDevice(ctx->device));
    SumScratch sc;
    sc.base = ctx->noalloc_scratch;
    sc.bytes = RBF_NOALLOC_SCRATCH_BYTES;
    return run_kernel_sum(ctx, pb, (hipStream_t)stream, &sc);
}

rbf_status rbf_evaluate(rbf_ctx ctx, int32_t dim, double radius, int64_t n_c, int64_t ld_ctrl,
                        const double *xc, const double *alpha, int64_t n_p, const double *xp,
                        const double *base, double sign, double *out, int32_t precision, int32_t basis,
                        void *stream)
{
    if (!ctx) return fail(RBF_E_INVALID, "ctx is NULL");
    if (dim != 2 && dim != 3) return fail(RBF_E_INVALID, "dim must be 2 or 3");
    if (!(radius > 0.0) || !std::isfinite(radius)) return fail(RBF_E_INVALID, "radius must be > 0");
    if (n_c < 0 || ld_ctrl < n_c) return fail(RBF_E_INVALID, "n_c/ld_ctrl out of range");
    if (n_p < 0 || n_p > (int64_t(1) << 31) - 1) return fail(RBF_E_INVALID, "n_p out of range");
    if (precision != RBF_FP64 && precision != RBF_MIXED) return fail(RBF_E_INVALID, "bad precision");
    if (!basis_valid(basis)) return fail(RBF_E_INVALID, "unknown basis %d", basis);
    if (!std::isfinite(sign)) return fail(RBF_E_INVALID, "sign must be finite");
    if (n_p == 0) return RBF_OK;
    if (!xp || !out || (n_c > 0 && (!xc || !alpha))) return fail(RBF_E_INVALID, "NULL device array");
    RBF_HIP(hipSetDevice(ctx->device));
    SumProblem pb;
    pb.dim = dim;
    pb.n_levels = 1;
    pb.lv[0] = SumLevel{1.0 / radius, 0.0, 0, n_c, precision == RBF_MIXED};
    pb.ld_ctrl = ld_ctrl;
    pb.xc = xc;
    pb.alpha = alpha;
    pb.n_p = n_p;
    pb.xp = xp;
    pb.base = base;
    pb.sign = sign;
    pb.out = out;
    pb.precision = precision;
    pb.basis = basis;
    return run_kernel_sum(ctx, pb, (hipStream_t)stream);
}

}  // extern "C"
