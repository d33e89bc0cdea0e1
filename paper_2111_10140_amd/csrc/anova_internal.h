// Internal declarations of the ANOVA fast-summation library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
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

// ---------------------------------------------------------------- device buffer
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ptr(o.ptr), bytes(o.bytes) { o.ptr = nullptr; o.bytes = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        release();
        ptr = o.ptr; bytes = o.bytes; o.ptr = nullptr; o.bytes = 0;
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t b) {
        release();
        if (b == 0) b = 256;
        ANOVA_HIP_CHECK(hipMalloc(&ptr, b));
        bytes = b;
    }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr; bytes = 0;
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
    const void *tmp;         // window's interpolated values, sorted order (float/double)
    const int32_t *iperm;    // caller's point index -> sorted position
    double eta;
};

// Degree of the per-offset window polynomials: the fit error of the
// Kaiser-Bessel window stays below 2e-7 (float32) and 1.2e-14 (float64) of
// its maximum for m = 2..8 and oversampling 1.25..4.
template <typename T> struct PolyDeg;
template <> struct PolyDeg<float> { static constexpr int value = 8; };
template <> struct PolyDeg<double> { static constexpr int value = 15; };

// ---------------------------------------------------------------- window plan
struct WindowPlan {
    // parameters
    int dA = 0, M = 0, n = 0, m = 0;
    int feat[3] = {0, 0, 0};
    double eta = 0, ell = 0, h = 0, extent = 0, kb_b = 0;
    double center[3] = {0, 0, 0};
    double err_images = 0, err_trunc = 0, err_window = 0, err_round = 0, err_total = 0;
    double fit_err = 0;          // max error of the window polynomials
    // tiling
    int tile = 0;                // tile edge in grid points (same in every dimension)
    int tiles_per_dim = 0;
    int64_t n_tiles = 0, n_nonempty = 0, n_sub = 0;
    int poly_deg = 0;
    bool dense = false;          // per-cell register accumulation (see kernels.hip)
    int chunks = 1;              // dense regime: workgroups per tile
    int64_t n_points = 0;
    int64_t n_regions = 0;       // spread regions per launch (sub-problems, or tiles x chunks)
    // device data
    DevBuf nodes;    // NodeF32 or NodeF64, sorted by tile (N entries)
    DevBuf perm;     // int32: sorted position -> caller's point index
    DevBuf iperm;    // int32: caller's point index -> sorted position
    DevBuf subs;     // SubProblem[n_sub]
    DevBuf poly;     // window polynomial table [2m][poly_deg+1] (float or double)
    DevBuf bconv;    // per-axis multiplier, n entries (float or double)
    DevBuf twiddle;  // n/2 complex exp(-2 pi i j / n) (float2 or double2)
    DevBuf src_sub;     // int32 [n_nonempty + 1]: spread regions of the k-th non-empty tile
    DevBuf cell_start;  // dense regime: int32 [cells + 1] sorted-point offsets per (tile, cell)
    DevBuf tiles_ne;    // dense regime: int32 ids of the non-empty tiles
    DevBuf fold_pairs;  // int2 {non-empty tile k, packed region offsets}, grouped by tile
    DevBuf fold_start;  // int32 [n_tiles + 1] offsets into fold_pairs
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

struct anova_plan_s {
    int64_t N = 0;
    int32_t d = 0;
    int32_t P = 0;
    int32_t precision = 0;
    double ell = 0;
    std::vector<anova::WindowPlan> win;
    // work space
    anova::DevBuf grid;      // largest window grid (float or double) x grid_slots
    anova::DevBuf priv;      // spread regions: max over windows of n_sub x region (float/double)
    anova::DevBuf treg;      // per-tile sums of the regions (windows whose tiles have several)
    anova::DevBuf asort;     // coefficients in a window's sorted order (float or double), N
    anova::DevBuf tmp;       // per-window interpolated values, P x N (float or double)
    anova::DevBuf combine;   // CombineWin[P]
    size_t grid_slot_elems = 0;
    int grid_slots = 0;
    int device = 0;
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

// kernel launchers (kernels.hip)
void launch_spread(const WindowPlan &w, int precision, const double *alpha, void *grid, void *as,
                   void *priv, void *treg, hipStream_t s);
void launch_spread_regions(const WindowPlan &w, int precision, const double *alpha, void *as,
                           void *priv, hipStream_t s);
void launch_fold(const WindowPlan &w, int precision, const void *priv, void *treg, void *grid,
                 hipStream_t s);
void launch_convolve(const WindowPlan &w, int precision, void *grid, hipStream_t s);
void launch_gather(const WindowPlan &w, int precision, const void *grid, void *tmp,
                   hipStream_t s);
void launch_combine(const void *wins, int P, int precision, const double *alpha, double *out,
                    double beta, int64_t N, bool accumulate, hipStream_t s);
void launch_zero(void *p, size_t bytes, hipStream_t s);

// one matvec of a plan for a single column (plan.hip)
void plan_matvec(anova_plan_s *p, const double *alpha, double *out, double beta, hipStream_t s);
void ensure_grid(anova_plan_s *p, int slots);

// stage kinds for the optional timing
enum StageKind {
    kStageFold = 0,
    kStageSpread = 1,
    kStageConvolve = 2,
    kStageGather = 3,
    kStageCombine = 4,
    kStageKinds = 5
};
// records an event pair around `launch` when the plan's timing is enabled
template <typename F>
void timed_launch(anova_plan_s *p, int kind, hipStream_t s, F &&launch);
hipEvent_t pool_event(anova_plan_s *p);

template <typename F>
void timed_launch(anova_plan_s *p, int kind, hipStream_t s, F &&launch) {
    if (!p->timing) {
        launch();
        return;
    }
    hipEvent_t a = pool_event(p), b = pool_event(p);
    ANOVA_HIP_CHECK(hipEventRecord(a, s));
    launch();
    ANOVA_HIP_CHECK(hipEventRecord(b, s));
    p->timed.push_back({kind, a, b});
}

}  // namespace anova
