// Internal declarations shared by the library's translation units: the context, its device
// pool, error plumbing and the kernel launchers. Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rbfdef.h"

namespace rbf {

// ---- errors ------------------------------------------------------------------------------------
void set_error(const char *fmt, ...);
rbf_status fail(rbf_status s, const char *fmt, ...);

#define RBF_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::rbf::fail(RBF_E_DEVICE, "%s failed: %s (%s:%d)", #call,                   \
                               hipGetErrorString(e_), __FILE__, __LINE__);                     \
    } while (0)

#define RBF_TRY(expr)                                                                          \
    do {                                                                                       \
        rbf_status s_ = (expr);                                                                \
        if (s_ < 0) return s_;                                                                 \
    } while (0)

// ---- device pool ---------------------------------------------------------------------------------
// Caching allocator bounded by the context's HBM budget. Blocks freed with free_after() stay
// unavailable until the work already enqueued on that stream has finished (stream-ordered reuse).
class Pool {
  public:
    Pool(int device, uint64_t budget) : device_(device), budget_(budget) {}
    ~Pool();
    rbf_status alloc(void **p, size_t bytes);
    void free_now(void *p);                       // caller guarantees no pending device use
    rbf_status free_after(void *p, hipStream_t s);  // reusable once s has passed this point
    uint64_t in_use() const { return held_; }
    uint64_t budget() const { return budget_; }
    uint64_t live() const { return live_; }

  private:
    void reclaim_locked();
    static size_t round_up(size_t b);
    int device_;
    uint64_t budget_;
    uint64_t held_ = 0;   // bytes obtained from hipMalloc and not yet returned to the driver
    uint64_t live_ = 0;   // bytes currently handed out
    std::mutex mu_;
    std::multimap<size_t, void *> free_;           // size -> block
    std::unordered_map<void *, size_t> size_of_;
    struct Deferred { void *p; hipEvent_t ev; };
    std::deque<Deferred> deferred_;
};

// RAII device buffer from the pool. A buffer obtained with get(pool, bytes, s) is bound to the
// stream s that its work is enqueued on: its destructor (an early return after some launches
// included) hands it back stream-ordered, so no other caller can receive it while kernels already
// enqueued on s may still use it. release_after() hands it back stream-ordered at once.
struct DevBuf {
    Pool *pool = nullptr;
    void *ptr = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : pool(o.pool), ptr(o.ptr), stream(o.stream), bound(o.bound) { o.ptr = nullptr; }
    ~DevBuf() { drop(); }
    void drop()
    {
        if (ptr && pool) {
            if (bound) (void)pool->free_after(ptr, stream);
            else pool->free_now(ptr);
        }
        ptr = nullptr;
    }
    rbf_status get(Pool *pl, size_t bytes)
    {
        drop();
        pool = pl;
        bound = false;
        return pl->alloc(&ptr, bytes);
    }
    rbf_status get(Pool *pl, size_t bytes, hipStream_t s)
    {
        drop();
        pool = pl;
        stream = s;
        bound = true;
        return pl->alloc(&ptr, bytes);
    }
    void release_after(hipStream_t s) {
        if (ptr && pool) (void)pool->free_after(ptr, s);
        ptr = nullptr;
    }
    void settle() { bound = false; }   // the caller waited for the stream: free at once
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

template <class... B> void settle_all(B &...b) { (b.settle(), ...); }

class Server;   // serving loop (serve.cpp)

// Newton basis and Cholesky factor of one greedy level, kept between requests on a geometry:
// V holds column j (basis function j at every surface point) tile by tile: for each tile of 64
// surface points, its n columns of 64 values are contiguous (pitch n). L is packed lower
// (row j at j (j + 1) / 2). They depend on the geometry, the radius and the control points only,
// so the next icing step warm-started from the same control points reuses them as they are.
struct LevelCache {
    DevBuf V, L;
    int64_t n = 0;          // control points (columns)
    double radius = 0.0;
    int32_t basis = RBF_WENDLAND_C2;
    std::vector<int64_t> ctrl;   // host copy, selection order
};

struct Geometry {
    int32_t dim = 0;
    int64_t n_s = 0, n_v = 0;
    // Volume stored in blocks of VBLOCK Z-ordered points, blocks by increasing smallest wall
    // distance; n_pad = whole blocks, padding slots have perm -1 and d = +inf.
    DevBuf xs, xv_sorted, d_sorted, perm;   // perm: stored slot -> caller's index
    DevBuf block_box;                       // [n_pad / BOXROWS][2 dim]: min, max of every BOXROWS stored points
    int64_t n_pad = 0;
    bool run_layout = false;                // runs of input points kept whole in the stored order
    std::vector<double> block_dmin;         // host: smallest wall distance of each stored block
    // Control sets of the last finished request (warm start), host copies per level.
    std::vector<std::vector<int64_t>> last_ctrl;
    std::vector<LevelCache> levels;   // resident Newton bases of the last finished request
    uint64_t cache_bytes = 0;         // device bytes held by `levels`
    // Orders in which the resident kernel sums take their row groups (heaviest first by the controls
    // each keeps, dealt across the compute units), one per launch shape, radii and support
    // distances. Entries live as long as the geometry, since a launch on another stream may still
    // read one.
    struct GroupOrder {
        int32_t P = 0, n_levels = 0;
        double inv_r[RBF_MAX_LEVELS]{}, D[RBF_MAX_LEVELS]{};
        DevBuf order;
    };
    std::mutex order_mu;
    std::vector<GroupOrder> orders;
    double last_use = 0.0;
    int32_t refs = 0;        // queued or running requests (guarded by the server's lock)
    bool running = false;    // a request on this geometry is running
    uint64_t bytes = 0;
};

}  // namespace rbf

namespace rbf {
// Optional per-kernel device timers (hipEvent pairs), resolved lazily when queried.
struct KernelTimers {
    std::mutex mu;
    bool enabled = false;
    bool count_pairs = false;
    struct Pending { std::string name; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare;   // resolved events, reused (no event creation per launch)
    hipEvent_t take();
    std::map<std::string, std::pair<double, int64_t>> total;   // name -> (ms, launches)
    // Evaluated-pair counters of the kernel sums, one device slot per timed kernel name.
    static constexpr int N_COUNT = 16;
    unsigned long long *dev_count = nullptr;
    std::map<std::string, int> slot;
    void begin(hipEvent_t *a, hipStream_t s);
    void end(const char *name, hipEvent_t a, hipStream_t s);
    // Two events for a kernel's own start and end (hipExtLaunchKernel), null while timing is
    // off; add() files them under name once the launch is enqueued.
    void pair(hipEvent_t *a, hipEvent_t *b);
    void add(const char *name, hipEvent_t a, hipEvent_t b);
    void resolve();
    unsigned long long *counter(const char *name);   // null while timing is off
    ~KernelTimers();
};
}  // namespace rbf

struct rbf_ctx_s {
    rbf::KernelTimers timers;
    int device = 0;
    hipDeviceProp_t prop{};
    std::unique_ptr<rbf::Pool> pool;
    rbf::Server *server = nullptr;   // created on first submit, deleted by server_shutdown
    std::mutex geom_mu;
    std::unordered_map<rbf_geom, std::unique_ptr<rbf::Geometry>> geoms;
    int n_cu = 256;
    void *noalloc_scratch = nullptr;   // this device's fixed scratch array (device address)
    // Co-residency budget of the persistent greedy kernels running at once (workgroups).
    std::mutex coop_mu;
    std::condition_variable coop_cv;
    int64_t coop_in_use = 0;
};

struct rbf_geom_s {};  // opaque handle; the address keys the context's geometry table

namespace rbf {

// ---- kernel sums (ksum.hip) ---------------------------------------------------------------------
// Points per stored volume block: one kernel-sum workgroup (256 lanes x 2 points).
constexpr int VBLOCK = 512;
// Stored points per kept bounding box (one wave of the resident kernel sum).
constexpr int BOXROWS = 64;

struct SumLevel {
    double inv_r;     // 1 / R_l
    double D;         // wall-distance support D_l, or 0 when psi is not applied
    int64_t c_begin;  // range in the packed control array
    int64_t c_end;
    int32_t fp32 = 0; // 1: this level's pair arithmetic in FP32 on shifted coordinates
};

struct SumProblem {
    int32_t dim = 3;
    int32_t n_levels = 1;
    SumLevel lv[RBF_MAX_LEVELS];
    int64_t ld_ctrl = 0;          // leading dimension of xc / alpha
    const double *xc = nullptr;   // [dim][ld_ctrl]
    const double *alpha = nullptr;
    int64_t n_p = 0;              // number of points
    const double *xp = nullptr;   // [dim][n_p]
    const double *dwall = nullptr;  // [n_p] or null (psi = 1)
    const double *base = nullptr;   // out = base - sign * sum (base null: 0)
    double sign = -1.0;
    double *out = nullptr;        // [dim][ld_out], fully written
    int64_t ld_out = 0;           // 0: n_p
    int32_t precision = RBF_FP64;
    int32_t basis = RBF_WENDLAND_C2;
    // Resident geometry: points (xp, dwall) are stored in blocks ordered by their smallest wall
    // distance, the reduced volume lies in the prefix [0, n_active), and the result of slot v goes
    // to out[.][perm[v]] (perm: stored -> caller order, -1 for padding); points with psi = 0 get
    // +0.0 through perm. n_active < 0: not used.
    const int32_t *perm = nullptr;
    int64_t n_active = -1;
    const double *block_box = nullptr;   // [n_pad / BOXROWS][2 dim] box of every BOXROWS stored points
    Geometry *geom = nullptr;            // resident geometry, whose cached row-group order the launch uses
};

// A caller's fixed device area for the scratch of one kernel sum (the allocation-free entry point).
struct SumScratch {
    void *base = nullptr;
    size_t bytes = 0;
};

// Enqueues the whole evaluation on `s`; scratch comes from the pool and is released
// stream-ordered, so the call does not wait for the device. With ext, the scratch is carved from
// ext instead (fewer control-list splits if their partial sums would not fit) and the call
// allocates nothing, records no timer events and counts no pairs.
rbf_status run_kernel_sum(rbf_ctx ctx, const SumProblem &pb, hipStream_t s, const SumScratch *ext = nullptr);

// ---- allocation-free entry point (noalloc.hip) ---------------------------------------------------
// Device address of the library's fixed scratch array on the current device.
rbf_status noalloc_scratch_address(void **ptr);

// ---- greedy (greedy.hip) ------------------------------------------------------------------------
// warm (optional): per-level resident Newton bases; a level whose seeds equal the cached control
// points (same radius) starts from the cached basis. Other levels with enough seeds form their
// basis from the blocked factor of the seeds' Phi_CC (seed_factor, seed_basis) instead of
// appending the seeds one at a time.
// store (optional): receives every level's basis after the call (best effort: a level whose copy
// cannot be allocated is left empty).
rbf_status run_greedy(rbf_ctx ctx, const rbf_greedy_params &p, int64_t n_s, const double *xs,
                      const double *ds, rbf_ctrl_set *out, hipStream_t s,
                      const std::vector<LevelCache> *warm = nullptr,
                      std::vector<LevelCache> *store = nullptr);
uint64_t cache_bytes(const std::vector<LevelCache> &levels, int64_t n_s);

// ---- dense solves (chol.hip) --------------------------------------------------------------------
rbf_status run_solve_weights(rbf_ctx ctx, int32_t dim, double radius, int64_t n_c,
                             const double *xc, const double *dsc, double *alpha, int32_t basis,
                             hipStream_t s);
// Seeded level start (launches only, stream-ordered). seed_factor: Phi_CC of the n points xc
// ([dim][n]) factored in place on A (row-major, lda = 64 ceil(n / 64), padding identity) by the
// blocked FP64 MFMA Cholesky, and dinv[kb] = inv(L_kb,kb) (row-major 64 x 64 blocks); a
// non-positive pivot sets *bad (device int32 the caller zeroed). seed_basis: Lpack = the factor's
// packed rows (row i at i (i + 1) / 2) and V = Phi_sC L^-T for the n_s surface points, written as
// columns 0..n-1 of the greedy's tile-major basis (64-point tiles, ldt columns per tile).
rbf_status seed_factor(int32_t dim, double radius, int32_t basis, int64_t n, const double *xc, double *A,
                       int64_t lda, double *dinv, int32_t *bad, hipStream_t s);
rbf_status seed_basis(int32_t dim, const double *xs, int64_t n_s, const double *xc, int64_t n, double radius,
                      int32_t basis, const double *A, int64_t lda, const double *dinv, double *V, int64_t ldt,
                      double *Lpack, hipStream_t s);

// ---- validation helpers (capi.cpp) ---------------------------------------------------------------
rbf_status validate_params(const rbf_greedy_params &p, int64_t n_s);
rbf_status check_precision(int32_t precision, const int32_t *level_precision, int32_t n_levels);
double now_seconds();

// ---- serving (serve.cpp) --------------------------------------------------------------------------
void server_shutdown(rbf_ctx ctx);   // stops the scheduler thread and drops its state
// Row-group order of a resident kernel sum with P points per lane over n_groups groups of 256 P
// stored rows: built on the first call for this shape, radii and support distances from that
// call's controls (one small kernel and a host sort), then reused by later calls with the same
// key whatever their controls (an order only decides which workgroup takes which group, never a
// result). *order is null when the cache is full.
rbf_status resident_order(rbf_ctx ctx, Geometry &g, const SumProblem &pb, int P, int64_t n_groups,
                          hipStream_t s, const int32_t **order);

}  // namespace rbf
