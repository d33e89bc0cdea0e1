// Internal declarations of the ANOVA fast-summation library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <memory>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/anova.h"

namespace anova {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
const char *get_error();

struct Error {
    anova_status st;
    std::string msg;
};

#define ANOVA_HIP_CHECK(expr)                                                              \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess)                                                              \
            throw ::anova::Error{_e == hipErrorOutOfMemory ? ANOVA_E_NOMEM : ANOVA_E_HIP,  \
                                 std::string(#expr) + ": " + hipGetErrorString(_e)};       \
    } while (0)

#define ANOVA_REQUIRE(cond, msg)                                                           \
    do {                                                                                   \
        if (!(cond)) throw ::anova::Error{ANOVA_E_INVALID, (msg)};                         \
    } while (0)

// Runs an entry point's body: a thrown Error becomes its status (message
// kept for anova_last_error), nothing else crosses the C ABI either.
template <typename F>
anova_status guarded(F &&f) {
    try {
        f();
        return ANOVA_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return ANOVA_E_NOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return ANOVA_E_HIP;
    }
}

// ---------------------------------------------------------------- device buffer
// Serialises the library's device allocations, frees and synchronous
// uploads with hipGraph captures, which other threads' such calls can
// invalidate (plans may be built on several host threads).
std::recursive_mutex &device_mutex();

// Small device blocks (tables of plans, batches and solves: up to
// kSmallBlockMax bytes, in power-of-two size classes) are kept per device
// for reuse when released instead of being freed: hipFree waits for the
// device, which stalls the work of other threads and streams (a serving
// loop frees and allocates such tables whenever a request starts or ends).
// A released block becomes reusable only after a device synchronisation
// that follows its release (one per many releases), as work queued before
// the release may still read it.  At most kSmallCacheBytes per device are
// kept.  Called with device_mutex() held; `dev` is the block's device.
constexpr size_t kSmallBlockMax = (size_t)1 << 20;
constexpr size_t kSmallCacheBytes = (size_t)256 << 20;
void *small_block_take(int dev, size_t cls);           // nullptr if none is cached
bool small_block_give(int dev, void *p, size_t cls);  // false: the cache is full

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int dev = -1;  // device of a cached-class block
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ptr(o.ptr), bytes(o.bytes), dev(o.dev) {
        o.ptr = nullptr; o.bytes = 0; o.dev = -1;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        release();
        ptr = o.ptr; bytes = o.bytes; dev = o.dev; o.ptr = nullptr; o.bytes = 0; o.dev = -1;
        return *this;
    }
    ~DevBuf() { release(); }
    static size_t size_class(size_t b) {
        size_t c = 256;
        while (c < b) c <<= 1;
        return c;
    }
    void alloc(size_t b) {
        release();
        if (b == 0) b = 256;
        std::lock_guard<std::recursive_mutex> lock(device_mutex());
        if (b <= kSmallBlockMax) {
            const size_t cls = size_class(b);
            int d = 0;
            ANOVA_HIP_CHECK(hipGetDevice(&d));
            ptr = small_block_take(d, cls);
            if (!ptr) ANOVA_HIP_CHECK(hipMalloc(&ptr, cls));
            bytes = cls;
            dev = d;
            return;
        }
        ANOVA_HIP_CHECK(hipMalloc(&ptr, b));
        bytes = b;
    }
    void release() {
        if (ptr) {
            std::lock_guard<std::recursive_mutex> lock(device_mutex());
            if (dev < 0 || !small_block_give(dev, ptr, bytes)) (void)hipFree(ptr);
        }
        ptr = nullptr; bytes = 0; dev = -1;
    }
    template <typename T> T *as() const { return static_cast<T *>(ptr); }
};

// ---------------------------------------------------------------- node records
// A point of one window after binning: fractional offsets inside its grid
// cell (in [0,1)) for each of the window's dimensions and the three cell
// indices packed as 10-bit fields (cell_x | cell_y << 10 | cell_z << 20).
struct alignas(16) NodeF32 {
    float f[3];
    uint32_t cell;
};
struct alignas(32) NodeF64 {
    double f[3];
    uint32_t cell;
    uint32_t pad;
};

// A spreading / gathering work item: one grid tile, a contiguous range of
// the tile's sorted points.
struct alignas(16) SubProblem {
    int32_t tile;     // linear tile index (x fastest)
    int32_t start;    // first sorted point
    int32_t count;    // number of points
    int32_t pad;
};

// Per-window operand of the combine kernel (device array, one per window).
struct CombineWin {
    const void *tmp;         // window's interpolated values, caller's order (float/double)
    double eta;
};

// Degree of the per-offset window polynomials of a support of W points: the
// fit error of the Kaiser-Bessel window stays below 2e-7 (float32: degree 8
// for m <= 2, 7 beyond) and 1.2e-14 (float64) of its maximum for m = 2..8
// and oversampling 1.25..4, and the plan counts it in the window error.
template <typename T> struct PolyDeg;
template <> struct PolyDeg<float> {
    static constexpr int of(int W) { return W <= 4 ? 8 : 7; }
};
template <> struct PolyDeg<double> {
    static constexpr int of(int) { return 15; }
};
// Degree of the float64 per-cell kernels' polynomials (3-D, W <= 6): those
// windows' own aliasing error is above 1e-8, and degree 11 fits to below
// 2e-10 of the maximum for m = 2, 3 and oversampling 1.25..4, with fewer
// scalar registers than degree 15 (the coefficients stay uniform).
constexpr int kPolyDegCell64 = 11;

// ---------------------------------------------------------------- window plan
struct WindowPlan {
    // parameters
    int dA = 0, M = 0, n = 0, m = 0;
    int feat[3] = {0, 0, 0};
    double eta = 0, ell = 0, h = 0, extent = 0, kb_b = 0;
    int reg_q = 0;               // > 0: regularised kernel, exact on [-extent, extent]
    double center[3] = {0, 0, 0};
    double err_images = 0, err_trunc = 0, err_window = 0, err_round = 0, err_total = 0;
    double fit_err = 0;          // max error of the window polynomials
    // tiling
    int tile = 0;                // tile edge in grid points (same in every dimension)
    int tile_cap = 0;            // > 0: per-point kernels take tiles of at most this
                                 // edge (the measured parameter choice tries halves)
    int tiles_per_dim = 0;
    int64_t n_tiles = 0, n_nonempty = 0, n_sub = 0;
    int poly_deg = 0;
    bool dense = false;          // per-cell register accumulation (see kernels.hip)
    int chunks = 1;              // dense regime: workgroups per tile
    int launch_windows = 1;      // windows whose launches share the device (the plan's)
    std::vector<int32_t> chunk_start;  // dense regime: first workgroup of each non-empty tile
    std::vector<int32_t> tile_order;   // dense regime: non-empty tiles in launch order
    int64_t n_points = 0;
    int64_t n_regions = 0;       // spread regions per launch (sub-problems, or tiles x chunks)
    // device data
    DevBuf nodes;    // NodeF32 or NodeF64, sorted by tile (N entries)
    DevBuf perm;     // int32: sorted position -> caller's point index
    DevBuf subs;     // SubProblem[n_sub]
    DevBuf poly;     // window polynomial table [2m][poly_deg+1] (float or double)
    DevBuf bconv;    // per-axis multiplier, n entries (float or double)
    DevBuf ctaps;    // its inverse transform: real, even circular-convolution taps, n entries
    DevBuf twiddle;  // n/2 complex exp(-2 pi i j / n) (float2 or double2)
    DevBuf src_sub;     // int32 [n_nonempty + 1]: spread regions of the k-th non-empty tile
    DevBuf cell_start;  // dense regime: int32 [cells + 1] sorted-point offsets per (tile, cell)
    DevBuf tiles_ne;    // dense regime: int32 ids of the non-empty tiles
    DevBuf fold_pairs;  // int2 {non-empty tile k, packed region offsets}, grouped by tile
    DevBuf fold_start;  // int32 [n_tiles + 1] offsets into fold_pairs
    DevBuf fold_tiles;  // int32 fold workgroup order: tiles with regions (die-grouped, -1
                        // padded to fold_act entries), then the tiles without
    int32_t fold_act = 0, fold_len = 0;
    int64_t n_pairs = 0;
    size_t region_elems() const {
        size_t L = (size_t)tile + 2 * m - 1, v = L;
        if (dA >= 2) v *= L;
        if (dA >= 3) v *= L;
        return v;
    }
    size_t grid_elems() const {
        size_t g = 1;
        for (int t = 0; t < dA; ++t) g *= (size_t)n;
        return g;
    }
};

}  // namespace anova

namespace anova {
class Batch;
}

struct anova_plan_s {
    int64_t N = 0;
    int32_t d = 0;
    int32_t P = 0;
    int32_t precision = 0;
    double ell = 0;
    std::vector<anova::WindowPlan> win;
    // float32 plans with float64 residuals: the same windows in float64
    // (empty otherwise)
    std::vector<anova::WindowPlan> win64;
    // prediction plans: the target points binned with each window's
    // parameters (empty otherwise)
    int64_t Nz = 0;
    std::vector<anova::WindowPlan> tgt;
    int device = 0;
    // batched launches of this plan's own products (anova_matvec) and
    // predictions (anova_predict), one per recently used set of vectors and
    // shift (least recently used last to be rebuilt)
    std::vector<std::unique_ptr<anova::Batch>> mv_cache, pred_cache;
    // optional per-stage timing (events on the launching stream)
    bool timing = false;
    struct TimedLaunch {
        int kind;
        hipEvent_t start, stop;
    };
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
};

namespace anova {

// ---------------------------------------------------------------- batched launches
// One window of one problem for one right-hand side, as seen by the kernels.
struct WinInst {
    const void *nodes;          // NodeF32 / NodeF64, sorted order
    const int32_t *perm;        // sorted position -> caller's index
    const SubProblem *subs;     // per-point mode work items
    const int32_t *tiles_ne;    // per-cell mode: non-empty tile ids
    const int32_t *cell_start;  // per-cell mode: point offsets per (tile, cell)
    const int32_t *src_sub;     // regions of each non-empty tile
    const int2 *fold_pairs;
    const int32_t *fold_start;
    const int32_t *fold_tiles;
    const void *poly;
    const void *bconv;
    const void *ctaps;
    const void *twiddle;
    const double *alpha;        // input column, caller's order
    void *priv;                 // spread regions
    void *treg;                 // per-tile region sums
    void *grid;                 // n^dA grid
    void *tmp;                  // sorted coefficients (per-point spread), then
                                // interpolated values in the caller's order
    int32_t n, tile, tpd, chunks;  // chunks: per-cell mode's workgroups per tile (every tile alike)
    int32_t vol, n_sub, n_nonempty, n_tiles;
    int32_t n_regions, N, dA, width;
    int32_t fold_act, fold_len;  // entries of fold_tiles: tiles with regions, all
};

// CG state of one column (device memory): the scalars of Sec. 2's
// conjugate-gradient recurrence and the column's stopping state.
struct CgScal {
    double rho;      // r.r of the current residual
    double ynorm2;   // y.y
    double tol2;     // tol^2
    double a, b;     // step length and direction update
    double pq;       // p.q of the current iteration
    int32_t active;  // 1 while the column iterates
    int32_t status;  // 0 running, 1 converged, 2 breakdown, 3 maxit reached
    int32_t iters;
    int32_t maxit;
    int32_t period;      // residual recomputed at iterations period, 2 period, ...
    int32_t exact_only;  // 1: stop only on a recomputed (float64) residual
};

// A product inside a CG iteration, q = (K~ + beta I) p: for each output
// column the combine kernel also forms the partial sums of p.q (one per
// combine workgroup of the column), so the iteration needs no separate pass
// over p and q for the step length.
struct CgHook {
    double *partial;
};

// One output column of the combine kernel.
struct CombInst {
    double *out;
    const double *alpha;
    double beta;
    int32_t N, win0, P, accumulate;
    CgHook hook;  // partial == nullptr: a plain product
};

// Stage identifiers; the first five are the reported timing kinds.
enum StageKind {
    kStagePermute = 0,
    kStageSpread = 1,
    kStageTileSum = 2,
    kStageFold = 3,
    kStageConvolve = 4,
    kStageGather = 5,
    kStageCombine = 6,
    kStageKinds = 7
};

// A launch: all instances of one stage sharing a kernel signature.
struct BatchGroup {
    int stage = 0;
    int cell = 0, dA = 0, W = 0, tile = 0, n = 0, axis = 0, np = 1;
    int blocks = 0, cnt = 0;
    const int32_t *members = nullptr;  // device: instance indices
    const int32_t *prefix = nullptr;   // device: block prefix (cnt + 1)
};

// Problem handed to a batch: a plan applied to nrhs columns.
struct BatchProblem {
    anova_plan_s *plan = nullptr;
    const double *alpha = nullptr;  // device, column-major, leading dimension ld
    double *out = nullptr;
    int nrhs = 1;
    int64_t ld = 0;                 // column stride of alpha
    int64_t ld_out = -1;            // column stride of out (-1: same as ld)
    double beta = 0.0;
    int only_window = -1;           // >= 0: stage entry points (one window)
    void *grid_override = nullptr;  // stage entry points: the caller's grid
    void *work = nullptr;           // problem_work_bytes() of work space owned by
                                    // the caller (nullptr: the batch allocates)
    bool residual = false;          // use the plan's float64 residual windows
                                    // when it has them
    bool predict = false;           // out (plan->Nz rows) = K~(Z, X) alpha: spread
                                    // at the plan's points, gather at its targets
    const CgHook *hooks = nullptr;  // host array of nrhs: the columns' CG
                                    // reductions fused into the combine
};

// Windows and arithmetic precision a batch problem runs with.
inline const std::vector<WindowPlan> &problem_windows(const BatchProblem &bp) {
    return bp.residual && !bp.plan->win64.empty() ? bp.plan->win64 : bp.plan->win;
}
inline int problem_precision(const BatchProblem &bp) {
    return bp.residual && !bp.plan->win64.empty() ? ANOVA_FP64 : bp.plan->precision;
}

// Work space (grids, spread regions, sorted values) of one problem's
// instances in a batch.
size_t problem_work_bytes(const BatchProblem &bp);
// Device bytes held by a plan's own buffers.
size_t plan_device_bytes(const anova_plan_s *p);

// Device memory a batch may use instead of allocating: its work space and
// launch tables are laid out from base, within bytes.
struct ExternalSpace {
    char *base;
    size_t bytes;
};

// A set of products run with one launch per stage and kernel signature.
class Batch {
  public:
    int precision = 0;
    std::vector<WinInst> insts;
    std::vector<uint8_t> roles;  // per instance: bit 0 spreads and convolves, bit 1 gathers
    std::vector<CombInst> combs;
    std::vector<CombineWin> cwins;
    std::vector<BatchGroup> groups;  // execution order
    DevBuf d_insts, d_combs, d_cwins, d_tables, work;
    int comb_blocks = 0, comb_cnt = 0;
    const int32_t *comb_prefix = nullptr;
    std::vector<BatchProblem> probs;

    // device addresses of the instance and combine tables (the batch's own
    // buffers, or inside the external space)
    const WinInst *dev_insts = nullptr;
    const CombInst *dev_combs = nullptr;
    const CombineWin *dev_cwins = nullptr;

    // (re)build for the given problems; workspace is reused when it fits.
    // With ext, nothing is allocated: work space and tables go into ext
    // (uploaded with synchronous copies; ANOVA_E_INVALID when they do not
    // fit), and the caller keeps ext's contents until the batch has run.
    void build(const std::vector<BatchProblem> &problems, const ExternalSpace *ext = nullptr);
    bool same(const std::vector<BatchProblem> &problems) const;
    // device bytes of the tables and of the batch-owned work space
    size_t device_bytes() const;
    // stage mask: bit k = stage kind k
    void run(hipStream_t s, anova_plan_s *timing = nullptr, unsigned mask = 0xffu) const;

    // A cached batch (a plan's own products) may be rebuilt in place for
    // other vectors.  The synchronous table uploads are not ordered after
    // work on the caller's stream, so a rebuild first waits for the batch's
    // last eager run; a batch that has run on a capturing stream is never
    // rebuilt (a graph holds its tables).
    void record_run(hipStream_t s);
    void wait_last_run();
    bool captured() const { return captured_; }
    Batch() = default;
    Batch(const Batch &) = delete;
    Batch &operator=(const Batch &) = delete;
    ~Batch();

  private:
    hipEvent_t last_run_ = nullptr;
    bool run_recorded_ = false;
    bool captured_ = false;
};

// Run the problems through a plan's cache of batches: the batch built for
// the same problems if there is one; else a new one while the cache holds
// fewer than kBatchCache, else the least recently used batch not captured
// by a graph, rebuilt after its last run has finished (a new one when every
// batch is captured).
constexpr size_t kBatchCache = 4;
void run_cached(std::vector<std::unique_ptr<Batch>> &cache, const std::vector<BatchProblem> &probs,
                hipStream_t s, anova_plan_s *timing);

// kernel-side entry points (kernels.hip)
void run_group(const BatchGroup &g, int precision, const WinInst *insts, hipStream_t s);
void run_combine(const CombInst *cis, const CombineWin *wins, const int32_t *prefix, int cnt,
                 int blocks, int precision, hipStream_t s);
int convolve_lines_per_block(int n, int nq, int elem_bytes);
int cell_tile(int dA);
bool cell_width_supported(int dA, int W, int precision);
int cell_point_splits(int dA, int W, int precision);
bool convolve_direct(int n, int dA);  // small grids: circular convolution by taps, planes then z
int cell_resident_blocks(int dA, int W, int precision);  // per-cell spreading workgroups held at once
int fold_blocks(const WinInst &w);  // fold workgroups of an instance
int combine_span();
int permute_span();

// plan helpers (plan.hip)
void plan_matvec(anova_plan_s *p, const double *alpha, double *out, int nrhs, int64_t ld,
                 double beta, hipStream_t s);
void plan_predict(anova_plan_s *p, const double *alpha, double *out, int nrhs, int64_t lda,
                  int64_t ldo, hipStream_t s);
template <typename T>
void upload(DevBuf &buf, const std::vector<T> &v) {
    size_t bytes = v.size() * sizeof(T);
    bytes = (bytes + 255) & ~(size_t)255;
    std::lock_guard<std::recursive_mutex> lock(device_mutex());
    if (!buf.ptr || buf.bytes < bytes) buf.alloc(bytes);
    if (!v.empty())
        ANOVA_HIP_CHECK(hipMemcpy(buf.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

// Points of a plan: rows of `ld` doubles in host memory (host != nullptr) or
// in device memory (dev != nullptr; kernels on stream s).
struct Points {
    const double *host = nullptr;
    const double *dev = nullptr;
    int64_t N = 0, ld = 0;
    hipStream_t s = nullptr;
};

// Device binning (binning.hip): per-point cells and offsets, the points'
// count per grid cell, and the sorted node records and permutation.
struct DeviceBins {
    DevBuf cellw, frac, hist, nodes, perm;
};
// Minimum and maximum of each of the d columns of device X; finite is
// false if some entry is not finite.  Synchronises s.
void device_bounds(const double *X, int64_t N, int64_t ld, int d, double *lo, double *hi,
                   bool &finite, hipStream_t s);
// Cells and offsets of every point of window w (its n, h, centre,
// features), and hist[cell] = points per grid cell (host copy).  Synchronises s.
template <typename T>
void device_bin(const double *X, int64_t N, int64_t ld, const WindowPlan &w, DeviceBins &b,
                std::vector<int32_t> &hist, hipStream_t s);
// Points sorted by (tile, cell inside the tile) when dense, else by tile,
// ties by original index: b.nodes (Node records) and b.perm.  Synchronises s.
template <typename T, typename Node>
void device_sort_nodes(const WindowPlan &w, int64_t N, int64_t cells_per_tile, bool dense,
                       DeviceBins &b, hipStream_t s);

// optional per-stage timing
hipEvent_t pool_event(anova_plan_s *p);
template <typename F>
void timed_launch(anova_plan_s *p, int kind, hipStream_t s, F &&launch) {
    if (!p || !p->timing) {
        launch();
        return;
    }
    hipEvent_t a = pool_event(p), b = pool_event(p);
    ANOVA_HIP_CHECK(hipEventRecord(a, s));
    launch();
    ANOVA_HIP_CHECK(hipEventRecord(b, s));
    p->timed.push_back({kind, a, b});
}

// ---------------------------------------------------------------- device loads
// A device pointer read from an instance record is generic to the compiler,
// so loads through it are flat loads, which also count against the LDS
// wait counter: waiting for an LDS read then waits for them too.  Loads
// through the global view are global loads, waited for on their own.
template <typename T>
using global_ptr = const __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ global_ptr<T> as_global(const T *p) {
    return (global_ptr<T>)p;
}
template <typename T>
using global_mut_ptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ global_mut_ptr<T> as_global_mut(T *p) {
    return (global_mut_ptr<T>)p;
}

// A zero in global memory: a lane with nothing to read loads it, so that
// loads need no condition and all of a batch go out before the first wait.
template <typename T>
__device__ const T kZeroValue = T(0);
template <typename T>
__device__ __forceinline__ T load_or_zero(global_ptr<T> p, bool ok) {
    return *(ok ? p : as_global(&kZeroValue<T>));
}

}  // namespace anova
