// Conjugate gradients for (K~ + beta I) alpha = y (Sec. 2: the system is
// symmetric positive definite for beta > 0 and is solved by CG with one
// kernel product per iteration; no preconditioner, Sec. 6).
//
// A solve (anova_cg_s) holds one problem's CG state for nrhs independent
// columns.  krr_cg_iterate advances any list of solves together: one
// iteration is a batched product over every (solve, window, column) followed
// by five vector kernels over the list of all columns, so problems of
// different sizes share each launch.  Everything except the product runs in
// float64: dot products are two-stage reductions (per-block partial sums,
// then one workgroup per column adding its partials in a fixed order, so
// results do not depend on scheduling), and the CG scalars stay in device
// memory, so an iteration needs no host round trip.  The iteration is
// captured once per solve list into a hipGraph and replayed.  At every
// period-th iteration of a column its recursive residual is replaced by
// y - A x (residual replacement); at the end the true residual is
// recomputed.  On float32 plans the replacement product is the float64 one
// (the plan's residual windows): the float32 product's rounding error grows
// with ||K|| and would otherwise stall the residual above tol for large N,
// so such a column stops only on a recomputed float64 residual.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <memory>
#include <mutex>

#include "anova_internal.h"

namespace anova {

constexpr int kRedBlock = 256;
constexpr int kSpan = 4 * kRedBlock;  // elements per block and column
constexpr int kResidualPeriod = 50;        // replacement with the plan's own product
constexpr int kResidualPeriodExact = 50;   // float64 residuals of float32 plans

// One column of one solve, as seen by the vector kernels.
struct CgCol {
    double *x;             // caller's alpha column
    double *r, *p, *q;
    const double *y;
    double *partial;       // nblk partial sums
    double *partial2;      // nblk partial sums of the replaced (recursive) residual
    CgScal *sc;
    double *cpartial;      // ncomb partial sums of p.q, written by the product's
                           // combine kernel
    int64_t N;
    int32_t nblk;
    int32_t ncomb;
};

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kRedBlock / 64; ++i) t += sh[i];
    __syncthreads();
    return t;  // valid in thread 0
}

__device__ __forceinline__ int find_col(const int32_t *__restrict__ prefix, int cnt, int b) {
    int lo = 0, hi = cnt;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// Block b of the column list: column c, element range [i0, i1).
struct ColRange {
    CgCol col;
    int lb;
    int64_t i0, i1;
};
__device__ __forceinline__ ColRange col_range(const CgCol *__restrict__ cols,
                                              const int32_t *__restrict__ prefix, int cnt) {
    const int c = find_col(prefix, cnt, blockIdx.x);
    ColRange r;
    r.col = cols[c];
    r.lb = blockIdx.x - prefix[c];
    r.i0 = (int64_t)r.lb * kSpan;
    r.i1 = min(r.col.N, r.i0 + kSpan);
    return r;
}

__device__ double sum_partials(const double *__restrict__ partial, int nblk, double *sh) {
    // a thread adds partials tid, tid + kRedBlock, ... in that order (a
    // missing one as +0), their loads issued eight at a time
    constexpr int B = 8;
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += B * kRedBlock) {
        double t[B];
#pragma unroll
        for (int u = 0; u < B; ++u) t[u] = load_or_zero(as_global(partial) + (i + u * kRedBlock), i + u * kRedBlock < nblk);
#pragma unroll
        for (int u = 0; u < B; ++u) v += t[u];
    }
    return block_sum(v, sh);
}

// ---------------------------------------------------------------- CG kernels
// x = 0, r = y, p = y, partial y.y
__global__ __launch_bounds__(kRedBlock) void cg_init_kernel(const CgCol *__restrict__ cols,
                                                            const int32_t *__restrict__ prefix,
                                                            int cnt) {
    __shared__ double sh[kRedBlock / 64];
    const ColRange cr = col_range(cols, prefix, cnt);
    double v = 0.0;
    for (int64_t i = cr.i0 + threadIdx.x; i < cr.i1; i += kRedBlock) {
        const double yi = cr.col.y[i];
        cr.col.x[i] = 0.0;
        cr.col.r[i] = yi;
        cr.col.p[i] = yi;
        v += yi * yi;
    }
    v = block_sum(v, sh);
    if (threadIdx.x == 0) cr.col.partial[cr.lb] = v;
}

__global__ __launch_bounds__(kRedBlock) void cg_init_scal_kernel(const CgCol *__restrict__ cols,
                                                                 double tol, int maxit,
                                                                 int period, int exact_only) {
    __shared__ double sh[kRedBlock / 64];
    const CgCol col = cols[blockIdx.x];
    const double y2 = sum_partials(col.partial, col.nblk, sh);
    if (threadIdx.x == 0) {
        CgScal s{};
        s.rho = y2;
        s.ynorm2 = y2;
        s.tol2 = tol * tol;
        s.active = (y2 > 0.0 && isfinite(y2)) ? 1 : 0;
        s.status = y2 > 0.0 ? (isfinite(y2) ? 0 : 2) : 1;
        s.iters = 0;
        s.maxit = maxit;
        s.period = period;
        s.exact_only = exact_only;
        *col.sc = s;
    }
}

// a = rho / (p.q), p.q from the partial sums of the product's combine kernel
__global__ __launch_bounds__(kRedBlock) void cg_alpha_kernel(const CgCol *__restrict__ cols) {
    __shared__ double sh[kRedBlock / 64];
    const CgCol col = cols[blockIdx.x];
    const double pq = sum_partials(col.cpartial, col.ncomb, sh);
    if (threadIdx.x == 0) {
        CgScal s = *col.sc;
        s.pq = pq;
        if (s.active) {
            if (pq == 0.0 && s.rho == 0.0) {
                s.a = 0.0;  // zero residual waiting for its float64 check
            } else if (!(pq > 0.0) || !isfinite(pq)) {
                s.active = 0;
                s.status = 2;
            } else {
                s.a = s.rho / pq;
            }
        }
        *col.sc = s;
    }
}

// rho' = r.r; convergence and iteration-limit tests; b = rho'/rho.
// `replaced`: this iteration recomputed the residual of the columns whose
// period is due (rr_rec: r.r of the recursive residual it replaced); an
// exact_only column may stop only then.  When such a recomputed (float64)
// residual has drifted above the recursive one (r.r more than 4 times
// larger), the float32 recursion has reached its rounding floor:
// continuing its directions would scale p by rho'/rho and the product's
// rounding with it, so the column restarts with p = r.
__device__ __forceinline__ void cg_direction_update(CgScal *sc, double rr, double rr_rec,
                                                    bool replaced) {
    CgScal s = *sc;
    if (s.active) {
        const bool now = replaced && (s.iters + 1) % s.period == 0;
        const bool checked = !s.exact_only || now;
        const bool restart = s.exact_only && now && rr > 4.0 * rr_rec;
        s.iters += 1;
        if (!isfinite(rr)) {
            s.active = 0;
            s.status = 2;
        } else if (checked && rr <= s.tol2 * s.ynorm2) {
            s.active = 0;
            s.status = 1;
            s.rho = rr;
        } else if (s.iters >= s.maxit) {
            s.active = 0;
            s.status = 3;
            s.rho = rr;
        } else {
            s.b = (s.rho > 0.0 && !restart) ? rr / s.rho : 0.0;
            s.rho = rr;
        }
    }
    *sc = s;
}

// x += a p; r -= a q; partial r.r
__global__ __launch_bounds__(kRedBlock) void cg_update_xr_kernel(const CgCol *__restrict__ cols,
                                                                 const int32_t *__restrict__ prefix,
                                                                 int cnt) {
    __shared__ double sh[kRedBlock / 64];
    const ColRange cr = col_range(cols, prefix, cnt);
    const CgScal sc = *cr.col.sc;
    double v = 0.0;
    for (int64_t i = cr.i0 + threadIdx.x; i < cr.i1; i += kRedBlock) {
        double ri = cr.col.r[i];
        if (sc.active) {
            cr.col.x[i] += sc.a * cr.col.p[i];
            ri -= sc.a * cr.col.q[i];
            cr.col.r[i] = ri;
        }
        v += ri * ri;
    }
    v = block_sum(v, sh);
    if (threadIdx.x == 0) cr.col.partial[cr.lb] = v;
}

// r = y - q (q = A x); partial r.r, and in partial2 the r.r of the
// recursive residual it replaces.  A column is replaced at its own
// iterations period, 2 period, ... (the current iteration is iters + 1), so
// the cadence does not depend on which other solves share the launch;
// `force` replaces every column (final residual).
__global__ __launch_bounds__(kRedBlock) void cg_replace_kernel(const CgCol *__restrict__ cols,
                                                               const int32_t *__restrict__ prefix,
                                                               int cnt, int force) {
    __shared__ double sh[kRedBlock / 64];
    const ColRange cr = col_range(cols, prefix, cnt);
    const CgScal sc = *cr.col.sc;
    const bool act = force || (sc.active != 0 && (sc.iters + 1) % sc.period == 0);
    double v = 0.0, v_rec = 0.0;
    for (int64_t i = cr.i0 + threadIdx.x; i < cr.i1; i += kRedBlock) {
        double ri = cr.col.r[i];
        if (act) {
            v_rec += ri * ri;
            ri = cr.col.y[i] - cr.col.q[i];
            cr.col.r[i] = ri;
        }
        v += ri * ri;
    }
    v = block_sum(v, sh);
    v_rec = block_sum(v_rec, sh);
    if (threadIdx.x == 0) {
        cr.col.partial[cr.lb] = v;
        cr.col.partial2[cr.lb] = v_rec;
    }
}

// The scalar update of an iteration (one workgroup per column): r.r of the
// residual and, when `replaced`, of the recursive one it replaced.
__global__ __launch_bounds__(kRedBlock) void cg_beta_kernel(const CgCol *__restrict__ cols,
                                                            int replaced) {
    __shared__ double sh[kRedBlock / 64];
    const CgCol col = cols[blockIdx.x];
    const double rr = sum_partials(col.partial, col.nblk, sh);
    const double rr_rec = replaced ? sum_partials(col.partial2, col.nblk, sh) : 0.0;
    if (threadIdx.x == 0) cg_direction_update(col.sc, rr, rr_rec, replaced != 0);
}

// p = r + b p
__global__ __launch_bounds__(kRedBlock) void cg_update_p_kernel(const CgCol *__restrict__ cols,
                                                                const int32_t *__restrict__ prefix,
                                                                int cnt) {
    const ColRange cr = col_range(cols, prefix, cnt);
    const CgScal sc = *cr.col.sc;
    if (!sc.active) return;
    for (int64_t i = cr.i0 + threadIdx.x; i < cr.i1; i += kRedBlock)
        cr.col.p[i] = cr.col.r[i] + sc.b * cr.col.p[i];
}

// Still-iterating columns of each solve of a list (solve s owns columns
// solve_cols[s] .. solve_cols[s+1]-1), one thread per solve.
__global__ __launch_bounds__(kRedBlock) void cg_active_kernel(const CgCol *__restrict__ cols,
                                                             const int32_t *__restrict__ solve_cols,
                                                             int count, int32_t *__restrict__ out) {
    const int s = blockIdx.x * kRedBlock + threadIdx.x;
    if (s >= count) return;
    int a = 0;
    for (int c = solve_cols[s]; c < solve_cols[s + 1]; ++c) a += cols[c].sc->active ? 1 : 0;
    out[s] = a;
}

// ---------------------------------------------------------------- column lists
struct ColList {
    std::vector<CgCol> cols;
    DevBuf d_cols, d_prefix;
    int blocks = 0, cnt = 0;
    void upload_lists() {
        std::vector<int32_t> prefix(cols.size() + 1, 0);
        for (size_t c = 0; c < cols.size(); ++c) prefix[c + 1] = prefix[c] + cols[c].nblk;
        blocks = prefix.back();
        cnt = (int)cols.size();
        upload(d_cols, cols);
        upload(d_prefix, prefix);
    }
};

}  // namespace anova

using namespace anova;

static std::atomic<uint64_t> g_next_solve_id{1};

struct anova_cg_s {
    anova_plan_s *plan = nullptr;
    uint64_t id = 0;
    int nrhs = 0;
    int64_t N = 0, ld = 0;
    const double *y = nullptr;
    double *x = nullptr;
    double beta = 1.0, tol = 0.0;
    int maxit = 0;
    int period = 0;           // residual replacement period
    bool exact_only = false;  // float32 plan with float64 residuals
    int64_t it = 0;  // iterations taken (every active column has taken as many)
    DevBuf r, p, q, partial, scal;
    DevBuf cpartial;  // p.q partials of the product's combine workgroups
    std::vector<CgHook> hooks;  // per column: where the combine puts them
    DevBuf work;  // product work space of this solve's (window, column) instances
    ColList own;  // this solve's columns alone (init, final residual)
    std::unique_ptr<Batch> xq;  // q = A x, for the final residual
};

namespace anova {

// Work space of one solve: its products p -> q (plan precision) and x -> q
// (residual windows) run one after another and share it.
static size_t solve_work_bytes(anova_plan_s *plan, int nrhs) {
    BatchProblem bp;
    bp.plan = plan;
    bp.nrhs = nrhs;
    const size_t a = problem_work_bytes(bp);
    bp.residual = true;
    return std::max(a, problem_work_bytes(bp));
}

// Captured iteration for one list of solves.
struct StepGraph {
    std::vector<uint64_t> ids;
    std::vector<anova_cg_s *> solves;
    ColList list;
    DevBuf d_solve_cols;  // int32 [count + 1]: first column of each solve in `list`
    Batch pq, xq;  // q = A p, q = A x over every solve in the list
    hipStream_t cap = nullptr;
    // one iteration, one with residual recomputation, kGraphIters
    // iterations without; each captured when first needed
    hipGraphExec_t g_plain = nullptr, g_replace = nullptr, g_block = nullptr;
    int64_t uses = 0;  // krr_cg_iterate calls on this list
    ~StepGraph() {
        if (g_plain) (void)hipGraphExecDestroy(g_plain);
        if (g_replace) (void)hipGraphExecDestroy(g_replace);
        if (g_block) (void)hipGraphExecDestroy(g_block);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

static std::mutex g_step_mu;
static std::vector<std::unique_ptr<StepGraph>> g_steps;  // small cache of captured lists
constexpr size_t kStepCache = 4;

static void record_iteration(StepGraph &G, bool replace, hipStream_t s) {
    const ColList &L = G.list;
    const CgCol *dc = L.d_cols.as<CgCol>();
    const int32_t *dp = L.d_prefix.as<int32_t>();
    // q = A p; the product's combine also forms the p.q partial sums
    G.pq.run(s);
    hipLaunchKernelGGL(cg_alpha_kernel, dim3(L.cnt), dim3(kRedBlock), 0, s, dc);
    hipLaunchKernelGGL(cg_update_xr_kernel, dim3(L.blocks), dim3(kRedBlock), 0, s, dc, dp, L.cnt);
    if (replace) {
        G.xq.run(s);
        hipLaunchKernelGGL(cg_replace_kernel, dim3(L.blocks), dim3(kRedBlock), 0, s, dc, dp, L.cnt,
                           0);
    }
    hipLaunchKernelGGL(cg_beta_kernel, dim3(L.cnt), dim3(kRedBlock), 0, s, dc, replace ? 1 : 0);
    hipLaunchKernelGGL(cg_update_p_kernel, dim3(L.blocks), dim3(kRedBlock), 0, s, dc, dp, L.cnt);
    ANOVA_HIP_CHECK(hipGetLastError());
}

static Batch &residual_batch(anova_cg_s *sv);

// An iteration in which only some solves of the list recompute their
// residual.  The others' columns would discard the product x -> q, so it
// runs for the due solves alone (each its own batch, as when it runs by
// itself); the launches are direct, since the due subset changes from one
// such iteration to the next.  The columns that are not due keep the r.r
// partials that the x, r update wrote, and the scalar update replaces
// only where the period is due, so every column takes the same steps as
// in a list whose members are all due or all not.
static void record_subset_replace(StepGraph &G, anova_cg_s *const *solves, int count,
                                  hipStream_t s) {
    const ColList &L = G.list;
    const CgCol *dc = L.d_cols.as<CgCol>();
    const int32_t *dp = L.d_prefix.as<int32_t>();
    G.pq.run(s);
    hipLaunchKernelGGL(cg_alpha_kernel, dim3(L.cnt), dim3(kRedBlock), 0, s, dc);
    hipLaunchKernelGGL(cg_update_xr_kernel, dim3(L.blocks), dim3(kRedBlock), 0, s, dc, dp, L.cnt);
    for (int i = 0; i < count; ++i) {
        anova_cg_s *sv = solves[i];
        if ((sv->it + 1) % sv->period != 0) continue;
        residual_batch(sv).run(s);
        hipLaunchKernelGGL(cg_replace_kernel, dim3(sv->own.blocks), dim3(kRedBlock), 0, s,
                           sv->own.d_cols.as<CgCol>(), sv->own.d_prefix.as<int32_t>(),
                           sv->own.cnt, 0);
    }
    hipLaunchKernelGGL(cg_beta_kernel, dim3(L.cnt), dim3(kRedBlock), 0, s, dc, 1);
    hipLaunchKernelGGL(cg_update_p_kernel, dim3(L.blocks), dim3(kRedBlock), 0, s, dc, dp, L.cnt);
    ANOVA_HIP_CHECK(hipGetLastError());
}

// Iterations replayed by one graph launch when none of them recomputes a
// residual: consecutive launches of separate graphs leave a gap of several
// microseconds between them, which a longer graph pays once.
constexpr int kGraphIters = 4;

static hipGraphExec_t capture(StepGraph &G, bool replace, int iters = 1) {
    hipGraph_t g = nullptr;
    ANOVA_HIP_CHECK(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
    try {
        for (int k = 0; k < iters; ++k) record_iteration(G, replace, G.cap);
    } catch (...) {
        (void)hipStreamEndCapture(G.cap, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    ANOVA_HIP_CHECK(hipStreamEndCapture(G.cap, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    ANOVA_HIP_CHECK(e);
    return ex;
}

// The graph of one iteration (replace: with residual recomputation) or of
// kGraphIters iterations (block), captured on first use.
static hipGraphExec_t graph_for(StepGraph &G, bool replace, bool block) {
    hipGraphExec_t &g = block ? G.g_block : (replace ? G.g_replace : G.g_plain);
    if (!g) {
        // capturing must not overlap other threads' allocations
        std::lock_guard<std::recursive_mutex> dev_lock(device_mutex());
        g = capture(G, replace, block ? kGraphIters : 1);
    }
    return g;
}

static BatchProblem product(anova_cg_s *sv, const double *in, bool residual) {
    BatchProblem bp;
    bp.residual = residual;
    bp.plan = sv->plan;
    bp.alpha = in;
    bp.out = sv->q.as<double>();
    bp.nrhs = sv->nrhs;
    bp.ld = sv->N;
    bp.beta = sv->beta;
    bp.work = sv->work.ptr;  // products of one solve run one after another on its stream
    return bp;
}

// The product q = (K~ + beta I) x of one solve alone (its residual
// recomputation), built on first use.
static Batch &residual_batch(anova_cg_s *sv) {
    if (!sv->xq) {
        BatchProblem bp = product(sv, sv->x, true);
        bp.ld = sv->ld;     // x columns follow the caller's leading dimension
        bp.ld_out = sv->N;  // q is packed
        std::unique_ptr<Batch> b(new Batch());
        b->build({bp});
        sv->xq = std::move(b);
    }
    return *sv->xq;
}

static StepGraph &step_graph(anova_cg_s *const *solves, int count) {
    // (the list cache is guarded by the caller's lock on the step mutex; a
    // hit takes no device lock, which planner threads hold while uploading)
    std::vector<uint64_t> ids(count);
    for (int i = 0; i < count; ++i) ids[i] = solves[i]->id;
    for (size_t k = 0; k < g_steps.size(); ++k)
        if (g_steps[k]->ids == ids) {
            std::unique_ptr<StepGraph> hit = std::move(g_steps[k]);
            g_steps.erase(g_steps.begin() + k);
            g_steps.push_back(std::move(hit));  // most recently used last
            return *g_steps.back();
        }
    // building and capturing must not overlap other threads' allocations
    std::lock_guard<std::recursive_mutex> dev_lock(device_mutex());
    std::unique_ptr<StepGraph> G(new StepGraph());
    G->ids = ids;
    G->solves.assign(solves, solves + count);
    std::vector<BatchProblem> pq_probs, xq_probs;
    std::vector<int32_t> solve_cols(1, 0);
    for (int i = 0; i < count; ++i) {
        anova_cg_s *sv = solves[i];
        G->list.cols.insert(G->list.cols.end(), sv->own.cols.begin(), sv->own.cols.end());
        solve_cols.push_back((int32_t)G->list.cols.size());
        BatchProblem bp = product(sv, sv->p.as<double>(), false);
        bp.hooks = sv->hooks.data();
        pq_probs.push_back(bp);
        BatchProblem bx = product(sv, sv->x, true);
        bx.ld = sv->ld;      // x columns follow the caller's leading dimension
        bx.ld_out = sv->N;   // q is packed
        xq_probs.push_back(bx);
    }
    G->list.upload_lists();
    upload(G->d_solve_cols, solve_cols);
    G->pq.build(pq_probs);
    G->xq.build(xq_probs);
    ANOVA_HIP_CHECK(hipStreamCreateWithFlags(&G->cap, hipStreamNonBlocking));
    if (g_steps.size() >= kStepCache) g_steps.erase(g_steps.begin());
    g_steps.push_back(std::move(G));
    return *g_steps.back();
}

static void drop_step_graphs(uint64_t id) {
    for (size_t k = 0; k < g_steps.size();) {
        if (std::find(g_steps[k]->ids.begin(), g_steps[k]->ids.end(), id) != g_steps[k]->ids.end())
            g_steps.erase(g_steps.begin() + k);
        else
            ++k;
    }
}

template <typename F>
static anova_status guarded_cg(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        set_error(e.msg);
        return e.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return ANOVA_E_NOMEM;
    }
}

static void fill_info(const anova_cg_s *sv, const std::vector<CgScal> &hs,
                      const std::vector<double> *true_rr, krr_cg_info *info) {
    for (int c = 0; c < sv->nrhs; ++c) {
        const CgScal &s = hs[c];
        info[c].iters = s.iters;
        info[c].converged = s.status == 1 ? 1 : 0;
        info[c].relres = s.ynorm2 > 0 ? std::sqrt(s.rho / s.ynorm2) : 0.0;
        info[c].true_relres =
            true_rr ? (s.ynorm2 > 0 ? std::sqrt((*true_rr)[c] / s.ynorm2) : 0.0) : info[c].relres;
    }
}

static std::vector<CgScal> read_scalars(const anova_cg_s *sv, hipStream_t s) {
    std::vector<CgScal> hs(sv->nrhs);
    ANOVA_HIP_CHECK(hipMemcpyAsync(hs.data(), sv->scal.ptr, sizeof(CgScal) * sv->nrhs,
                                   hipMemcpyDeviceToHost, s));
    ANOVA_HIP_CHECK(hipStreamSynchronize(s));
    return hs;
}

}  // namespace anova

extern "C" anova_status krr_cg_start(anova_cg_t *out, anova_plan_t plan, const double *y,
                                     double *alpha, int32_t nrhs, int64_t ld, double beta,
                                     double tol, int32_t maxit, void *stream) {
    if (!out) {
        set_error("out is NULL");
        return ANOVA_E_INVALID;
    }
    *out = nullptr;
    return guarded_cg([&] {
        ANOVA_REQUIRE(plan != nullptr, "NULL plan");
        ANOVA_REQUIRE(y != nullptr && alpha != nullptr, "NULL vector");
        ANOVA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        ANOVA_REQUIRE(ld >= plan->N, "ld must be >= N");
        ANOVA_REQUIRE(std::isfinite(beta) && beta > 0, "beta must be finite and > 0");
        ANOVA_REQUIRE(std::isfinite(tol) && tol >= 0, "tol must be finite and >= 0");
        ANOVA_REQUIRE(maxit >= 1, "maxit must be >= 1");
        hipStream_t s = (hipStream_t)stream;
        std::unique_ptr<anova_cg_s> sv(new anova_cg_s());
        sv->plan = plan;
        sv->id = g_next_solve_id++;
        sv->nrhs = nrhs;
        sv->N = plan->N;
        sv->ld = ld;
        sv->y = y;
        sv->x = alpha;
        sv->beta = beta;
        sv->tol = tol;
        sv->maxit = maxit;
        const int nblk = (int)((sv->N + kSpan - 1) / kSpan);
        const size_t vec = (size_t)sv->N * nrhs * sizeof(double);
        sv->r.alloc(vec);
        sv->p.alloc(vec);
        sv->q.alloc(vec);
        sv->partial.alloc((size_t)2 * nblk * nrhs * sizeof(double));
        sv->scal.alloc(sizeof(CgScal) * nrhs);
        const int64_t ncomb = (sv->N + combine_span() - 1) / combine_span();
        sv->cpartial.alloc((size_t)ncomb * nrhs * sizeof(double));
        sv->exact_only = plan->precision == ANOVA_FP32_NFFT && !plan->win64.empty();
        sv->period = sv->exact_only ? kResidualPeriodExact : kResidualPeriod;
        sv->work.alloc(solve_work_bytes(plan, nrhs));
        for (int c = 0; c < nrhs; ++c) {
            CgCol col{};
            col.x = alpha + (size_t)c * ld;
            col.r = sv->r.as<double>() + (size_t)c * sv->N;
            col.p = sv->p.as<double>() + (size_t)c * sv->N;
            col.q = sv->q.as<double>() + (size_t)c * sv->N;
            col.y = y + (size_t)c * ld;
            col.partial = sv->partial.as<double>() + (size_t)c * nblk;
            col.partial2 = sv->partial.as<double>() + (size_t)(nrhs + c) * nblk;
            col.sc = sv->scal.as<CgScal>() + c;
            col.cpartial = sv->cpartial.as<double>() + (size_t)c * ncomb;
            col.ncomb = (int32_t)ncomb;
            sv->hooks.push_back(CgHook{col.cpartial});
            col.N = sv->N;
            col.nblk = nblk;
            sv->own.cols.push_back(col);
        }
        sv->own.upload_lists();
        const CgCol *dc = sv->own.d_cols.as<CgCol>();
        hipLaunchKernelGGL(cg_init_kernel, dim3(sv->own.blocks), dim3(kRedBlock), 0, s, dc,
                           sv->own.d_prefix.as<int32_t>(), sv->own.cnt);
        hipLaunchKernelGGL(cg_init_scal_kernel, dim3(sv->own.cnt), dim3(kRedBlock), 0, s, dc, tol,
                           maxit, sv->period, sv->exact_only ? 1 : 0);
        ANOVA_HIP_CHECK(hipGetLastError());
        *out = sv.release();
        return ANOVA_OK;
    });
}

extern "C" anova_status krr_cg_iterate(anova_cg_t *solves, int32_t count, int32_t iters,
                                       void *stream) {
    return guarded_cg([&] {
        ANOVA_REQUIRE(solves != nullptr && count >= 1, "empty solve list");
        ANOVA_REQUIRE(iters >= 0, "iters must be >= 0");
        for (int i = 0; i < count; ++i) {
            ANOVA_REQUIRE(solves[i] != nullptr, "NULL solve");
            for (int j = 0; j < i; ++j) ANOVA_REQUIRE(solves[j] != solves[i], "repeated solve");
            ANOVA_REQUIRE(solves[i]->plan->precision == solves[0]->plan->precision &&
                              solves[i]->exact_only == solves[0]->exact_only,
                          "solves of one list must share the precision and residual mode");
        }
        std::lock_guard<std::mutex> lock(g_step_mu);
        StepGraph &G = step_graph(solves, count);
        hipStream_t s = (hipStream_t)stream;
        // a list's first call launches its iterations directly: the lists
        // of a serving loop change as requests join and leave, and one
        // used once would not repay the captures
        const bool direct = G.uses++ == 0;
        for (int k = 0; k < iters;) {
            // the next kGraphIters iterations in one launch when no solve
            // recomputes its residual in them
            bool block = iters - k >= kGraphIters;
            for (int i = 0; i < count && block; ++i)
                for (int j = 1; j <= kGraphIters; ++j)
                    block = block && (solves[i]->it + j) % solves[i]->period != 0;
            if (block) {
                if (direct)
                    for (int j = 0; j < kGraphIters; ++j) record_iteration(G, false, s);
                else
                    ANOVA_HIP_CHECK(hipGraphLaunch(graph_for(G, false, true), s));
                for (int i = 0; i < count; ++i) solves[i]->it += kGraphIters;
                k += kGraphIters;
                continue;
            }
            bool rep = false, all_due = true;
            for (int i = 0; i < count; ++i) {
                const bool due = (solves[i]->it + 1) % solves[i]->period == 0;
                rep = rep || due;
                all_due = all_due && due;
            }
            if (rep && !all_due)
                record_subset_replace(G, solves, count, s);
            else if (direct)
                record_iteration(G, rep, s);
            else
                ANOVA_HIP_CHECK(hipGraphLaunch(graph_for(G, rep, false), s));
            for (int i = 0; i < count; ++i) ++solves[i]->it;
            ++k;
        }
        return ANOVA_OK;
    });
}

extern "C" anova_status krr_cg_poll(anova_cg_t sv, int32_t *active, krr_cg_info *info,
                                    void *stream) {
    return guarded_cg([&] {
        ANOVA_REQUIRE(sv != nullptr, "NULL solve");
        const std::vector<CgScal> hs = read_scalars(sv, (hipStream_t)stream);
        int a = 0;
        for (auto &c : hs) a += c.active ? 1 : 0;
        if (active) *active = a;
        if (info) fill_info(sv, hs, nullptr, info);
        return ANOVA_OK;
    });
}

extern "C" anova_status krr_cg_active(anova_cg_t *solves, int32_t count, int32_t *dev_counts,
                                      int32_t *host_counts, void *stream) {
    return guarded_cg([&] {
        ANOVA_REQUIRE(solves != nullptr && count >= 1, "empty solve list");
        ANOVA_REQUIRE(dev_counts != nullptr && host_counts != nullptr, "NULL count array");
        for (int i = 0; i < count; ++i) ANOVA_REQUIRE(solves[i] != nullptr, "NULL solve");
        std::lock_guard<std::mutex> lock(g_step_mu);
        StepGraph &G = step_graph(solves, count);
        hipStream_t s = (hipStream_t)stream;
        hipLaunchKernelGGL(cg_active_kernel, dim3((count + kRedBlock - 1) / kRedBlock),
                           dim3(kRedBlock), 0, s, G.list.d_cols.as<CgCol>(),
                           G.d_solve_cols.as<int32_t>(), count, dev_counts);
        ANOVA_HIP_CHECK(hipGetLastError());
        ANOVA_HIP_CHECK(hipMemcpyAsync(host_counts, dev_counts, sizeof(int32_t) * count,
                                       hipMemcpyDeviceToHost, s));
        return ANOVA_OK;
    });
}

extern "C" anova_status krr_cg_finish(anova_cg_t sv, krr_cg_info *info, void *stream) {
    return guarded_cg([&] {
        ANOVA_REQUIRE(sv != nullptr, "NULL solve");
        hipStream_t s = (hipStream_t)stream;
        // true residual r = y - (K~ + beta I) x for every column
        residual_batch(sv).run(s);
        hipLaunchKernelGGL(cg_replace_kernel, dim3(sv->own.blocks), dim3(kRedBlock), 0, s,
                           sv->own.d_cols.as<CgCol>(), sv->own.d_prefix.as<int32_t>(),
                           sv->own.cnt, 1);
        ANOVA_HIP_CHECK(hipGetLastError());
        const int nblk = sv->own.cols.empty() ? 0 : sv->own.cols[0].nblk;
        std::vector<double> part((size_t)nblk * sv->nrhs);
        ANOVA_HIP_CHECK(hipMemcpyAsync(part.data(), sv->partial.ptr, part.size() * sizeof(double),
                                       hipMemcpyDeviceToHost, s));
        const std::vector<CgScal> hs = read_scalars(sv, s);
        std::vector<double> trr(sv->nrhs, 0.0);
        for (int c = 0; c < sv->nrhs; ++c)
            for (int b = 0; b < nblk; ++b) trr[c] += part[(size_t)c * nblk + b];
        if (info) fill_info(sv, hs, &trr, info);
        bool all_conv = true, breakdown = false;
        for (auto &c : hs) {
            all_conv = all_conv && c.status == 1;
            breakdown = breakdown || c.status == 2;
        }
        if (breakdown) {
            set_error("CG breakdown (p^T A p <= 0 or a non-finite value)");
            return ANOVA_E_BREAKDOWN;
        }
        if (!all_conv) {
            set_error("CG reached maxit before the tolerance");
            return ANOVA_E_NOT_CONVERGED;
        }
        return ANOVA_OK;
    });
}

extern "C" anova_status krr_cg_destroy(anova_cg_t sv) {
    if (!sv) return ANOVA_OK;
    return guarded_cg([&] {
        {
            std::lock_guard<std::mutex> lock(g_step_mu);
            drop_step_graphs(sv->id);
        }
        (void)hipDeviceSynchronize();
        delete sv;
        return ANOVA_OK;
    });
}

extern "C" anova_status anova_plan_footprint(anova_plan_t plan, int32_t nrhs,
                                             int64_t *plan_bytes, int64_t *solve_bytes) {
    return guarded_cg([&] {
        ANOVA_REQUIRE(plan != nullptr, "NULL plan");
        ANOVA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        if (plan_bytes) *plan_bytes = (int64_t)plan_device_bytes(plan);
        if (solve_bytes) {
            const int64_t N = plan->N;
            const int64_t nblk = (N + kSpan - 1) / kSpan;
            // r, p, q, partial sums, scalars, work space, column tables
            // (each allocation rounded as DevBuf rounds it: small blocks to
            // their size class)
            auto dev = [](size_t b) {
                if (b == 0) b = 256;
                return (int64_t)(b <= kSmallBlockMax ? DevBuf::size_class(b) : b);
            };
            int64_t b = 3 * dev((size_t)N * nrhs * sizeof(double));
            b += dev((size_t)2 * nblk * nrhs * sizeof(double)) + dev(sizeof(CgScal) * nrhs);
            const int64_t ncomb = (N + combine_span() - 1) / combine_span();
            b += dev((size_t)ncomb * nrhs * sizeof(double));
            b += dev(solve_work_bytes(plan, nrhs));
            b += dev(sizeof(CgCol) * nrhs) + dev(sizeof(int32_t) * (nrhs + 1));
            *solve_bytes = b;
        }
        return ANOVA_OK;
    });
}

static anova_status solve_lists(int32_t count, anova_cg_t *svs, int32_t check_every,
                                void *stream) {
    // iterate until no column is active, reading every solve's count of
    // active columns every few steps (one kernel and one copy for the list).
    // Columns that stop only on a recomputed residual (one list shares the
    // residual mode) can stop only at their period or at maxit, so their
    // counts are read there.
    return guarded_cg([&]() -> anova_status {
        std::vector<anova_cg_t> live(svs, svs + count);
        DevBuf dev_counts;
        dev_counts.alloc(sizeof(int32_t) * (size_t)count);
        std::vector<int32_t> act(count);
        while (!live.empty()) {
            const int32_t n = (int32_t)live.size();
            int64_t iters = check_every;
            if (live[0]->exact_only) {
                iters = INT64_MAX;
                for (anova_cg_t sv : live) {
                    iters = std::min<int64_t>(iters, sv->period - sv->it % sv->period);
                    if (sv->maxit > sv->it) iters = std::min<int64_t>(iters, sv->maxit - sv->it);
                }
            }
            anova_status st = krr_cg_iterate(live.data(), n, (int32_t)iters, stream);
            if (st == ANOVA_OK)
                st = krr_cg_active(live.data(), n, dev_counts.as<int32_t>(), act.data(), stream);
            if (st != ANOVA_OK) return st;
            ANOVA_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
            std::vector<anova_cg_t> still;
            for (int32_t i = 0; i < n; ++i)
                if (act[i] > 0) still.push_back(live[i]);
            live.swap(still);
        }
        return ANOVA_OK;
    });
}

extern "C" anova_status krr_cg_solve(anova_plan_t plan, const double *y, double *alpha,
                                     int32_t nrhs, int64_t ld, double beta, double tol,
                                     int32_t maxit, krr_cg_info *info, void *stream) {
    anova_cg_t sv = nullptr;
    anova_status st = krr_cg_start(&sv, plan, y, alpha, nrhs, ld, beta, tol, maxit, stream);
    if (st != ANOVA_OK) return st;
    st = solve_lists(1, &sv, 8, stream);
    if (st == ANOVA_OK) st = krr_cg_finish(sv, info, stream);
    const std::string msg = st != ANOVA_OK ? anova_last_error() : "";
    krr_cg_destroy(sv);
    if (st != ANOVA_OK) set_error(msg);
    return st;
}

extern "C" anova_status krr_cg_solve_batched(int32_t count, const anova_plan_t *plans,
                                             const double *const *y, double *const *alpha,
                                             const int32_t *nrhs, const int64_t *ld,
                                             const double *beta, double tol, int32_t maxit,
                                             krr_cg_info *info, void *stream) {
    if (count < 1 || !plans || !y || !alpha || !nrhs || !ld || !beta) {
        set_error("invalid batched solve arguments");
        return ANOVA_E_INVALID;
    }
    std::vector<anova_cg_t> svs(count, nullptr);
    anova_status st = ANOVA_OK;
    for (int i = 0; i < count && st == ANOVA_OK; ++i)
        st = krr_cg_start(&svs[i], plans[i], y[i], alpha[i], nrhs[i], ld[i], beta[i], tol, maxit,
                          stream);
    if (st == ANOVA_OK) st = solve_lists(count, svs.data(), 8, stream);
    anova_status worst = st;
    std::string msg = st != ANOVA_OK ? anova_last_error() : "";
    int64_t off = 0;
    for (int i = 0; i < count && st == ANOVA_OK; ++i) {
        const anova_status fi = krr_cg_finish(svs[i], info ? info + off : nullptr, stream);
        off += nrhs[i];
        if (fi != ANOVA_OK && (worst == ANOVA_OK || worst == ANOVA_E_NOT_CONVERGED)) {
            worst = fi;
            msg = anova_last_error();
        }
    }
    for (anova_cg_t sv : svs) krr_cg_destroy(sv);
    if (worst != ANOVA_OK) set_error(msg);
    return worst;
}
