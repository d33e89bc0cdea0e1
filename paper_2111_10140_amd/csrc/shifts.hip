// Conjugate gradients for several regularisation parameters at once:
// (K~ + lambda_s I) alpha_s = y for s = 0..S-1 (the lambda grid of the
// paper's grid search, Sec. 6; each system is the normal equation of Sec. 2).
//
// The systems differ by multiples of the identity, so they share one Krylov
// space: CG on the base system A_0 = K~ + lambda_min I produces residuals
// r_k, and the residual of the shifted system A_0 + sigma_s I after k steps
// is the collinear zeta_s,k r_k.  Requiring this collinearity in the CG
// recurrences (x_{k+1} = x_k + a_k p_k, r_{k+1} = r_k - a_k A p_k,
// p_{k+1} = r_{k+1} + b_k p_k for every system) gives, with
// zeta_0 = zeta_{-1} = 1, a_{-1} = 1, b_{-1} = 0:
//   zeta_{k+1} = zeta_k zeta_{k-1} a_{k-1} /
//                (a_k b_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} a_{k-1} (1 + sigma a_k))
//   a^s_k = a_k zeta_{k+1} / zeta_k,  b^s_k = (zeta_{k+1} / zeta_k)^2 b_k
//   x^s += a^s_k p^s,                 p^s = zeta_{k+1} r_{k+1} + b^s_k p^s
// (the shifted-CG recurrences of Frommer and Maass and of Jegerlehner).
// One kernel product per iteration serves every shift; each shift adds two
// float64 vector updates.  A shift stops when its residual |zeta| ||r||
// reaches tol ||y||.
//
// The recurrences hold in exact arithmetic for the operator the product
// applies.  On float32 plans that product's rounding separates the true and
// recursive residuals at large N (the reason single-shift CG replaces its
// residual), and a replaced residual would not be collinear any more.  So
// after the shared iterations every shift's true residual y - (K~ +
// lambda_s I) x_s is computed with the float64 product, and a shift that
// misses tol is refined: krr_cg_solve on that residual, whose solution is
// added to x_s.
#include <algorithm>
#include <cmath>
#include <vector>

#include "anova_internal.h"

namespace anova {

namespace {

constexpr int kMsBlock = 256;
constexpr int kMsSpan = 4 * kMsBlock;  // elements per block
constexpr int kMaxShifts = 32;
constexpr int kCheckEvery = 8;  // iterations between host checks for completion

struct MsShift {
    double *x;        // caller's solution column
    double *p;        // search direction (shift 0 is the base system's)
    double sigma;     // lambda_s - lambda_min
    double zeta, zeta_prev;
    double as, bs;    // this iteration's a^s, b^s
    double res2;      // zeta^2 r.r after the latest update
    int32_t active;   // 1 while the shift iterates
    int32_t upd;      // 1: apply this iteration's x update
    int32_t iters;    // shared iterations this shift took part in
    int32_t pad;
};

struct MsState {
    double rr;        // r.r of the base residual
    double ynorm2, tol2;
    double a, a_prev, b, b_prev;
    int32_t iters, maxit;
    int32_t status;   // 0 running, 1 all shifts converged, 2 breakdown, 3 maxit
    int32_t any;      // some shift still iterates
    int32_t apply;    // 1: the shift updates of this iteration are due (set by
                      // the shift scalars, cleared at the start of the next
                      // iteration, so launches after the end change nothing)
    int32_t pad;
};

__device__ __forceinline__ double ms_block_sum(double v, double *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kMsBlock / 64; ++i) t += sh[i];
    __syncthreads();
    return t;  // valid in thread 0
}

// fixed-order sum of nblk partials (one workgroup)
__device__ double ms_sum_partials(const double *__restrict__ partial, int nblk, double *sh) {
    // partials tid, tid + kMsBlock, ... in that order (a missing one as +0),
    // their loads issued eight at a time
    constexpr int B = 8;
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += B * kMsBlock) {
        double t[B];
#pragma unroll
        for (int u = 0; u < B; ++u) t[u] = load_or_zero(as_global(partial) + (i + u * kMsBlock), i + u * kMsBlock < nblk);
#pragma unroll
        for (int u = 0; u < B; ++u) v += t[u];
    }
    return ms_block_sum(v, sh);
}

// r = y, every p^s = y, every x^s = 0; partial y.y
__global__ __launch_bounds__(kMsBlock) void ms_init_kernel(const double *__restrict__ y,
                                                           double *__restrict__ r,
                                                           const MsShift *__restrict__ sh_tab,
                                                           int S, int64_t N,
                                                           double *__restrict__ partial) {
    __shared__ double sh[kMsBlock / 64];
    const int64_t i0 = (int64_t)blockIdx.x * kMsSpan;
    const int64_t i1 = min(N, i0 + kMsSpan);
    double v = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kMsBlock) {
        const double yi = y[i];
        r[i] = yi;
        for (int s = 0; s < S; ++s) {
            sh_tab[s].x[i] = 0.0;
            sh_tab[s].p[i] = yi;
        }
        v += yi * yi;
    }
    v = ms_block_sum(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

__global__ __launch_bounds__(kMsBlock) void ms_init_scal_kernel(MsShift *__restrict__ sh_tab, int S,
                                                                MsState *__restrict__ st,
                                                                const double *__restrict__ partial,
                                                                int nblk, double tol, int maxit) {
    __shared__ double sh[kMsBlock / 64];
    const double y2 = ms_sum_partials(partial, nblk, sh);
    if (threadIdx.x == 0) {
        MsState t{};
        t.rr = y2;
        t.ynorm2 = y2;
        t.tol2 = tol * tol;
        t.a = 0.0;
        t.a_prev = 1.0;
        t.b = 0.0;
        t.b_prev = 0.0;
        t.iters = 0;
        t.maxit = maxit;
        const bool run = y2 > 0.0 && isfinite(y2);
        t.status = run ? 0 : (y2 > 0.0 ? 2 : 1);
        t.any = run ? 1 : 0;
        *st = t;
        for (int s = 0; s < S; ++s) {
            MsShift &e = sh_tab[s];
            e.zeta = 1.0;
            e.zeta_prev = 1.0;
            e.as = 0.0;
            e.bs = 0.0;
            e.res2 = y2;
            e.active = run ? 1 : 0;
            e.upd = 0;
            e.iters = 0;
        }
    }
}

// partial p^0 . q; clears the previous iteration's update flag
__global__ __launch_bounds__(kMsBlock) void ms_dot_kernel(const double *__restrict__ p,
                                                          const double *__restrict__ q, int64_t N,
                                                          MsState *__restrict__ st,
                                                          double *__restrict__ partial) {
    __shared__ double sh[kMsBlock / 64];
    if (blockIdx.x == 0 && threadIdx.x == 0) st->apply = 0;  // read by no other block here
    if (!st->any) return;
    const int64_t i0 = (int64_t)blockIdx.x * kMsSpan;
    const int64_t i1 = min(N, i0 + kMsSpan);
    double v = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kMsBlock) v += p[i] * q[i];
    v = ms_block_sum(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// a = rr / (p.q), or breakdown
__global__ __launch_bounds__(kMsBlock) void ms_alpha_kernel(MsState *__restrict__ st,
                                                            const double *__restrict__ partial,
                                                            int nblk) {
    __shared__ double sh[kMsBlock / 64];
    if (!st->any) return;
    const double pq = ms_sum_partials(partial, nblk, sh);
    if (threadIdx.x == 0) {
        if (!(pq > 0.0) || !isfinite(pq)) {
            st->any = 0;
            st->status = 2;
        } else {
            st->a = st->rr / pq;
        }
    }
}

// r -= a q; partial r.r
__global__ __launch_bounds__(kMsBlock) void ms_update_r_kernel(double *__restrict__ r,
                                                               const double *__restrict__ q,
                                                               int64_t N,
                                                               const MsState *__restrict__ st,
                                                               double *__restrict__ partial) {
    __shared__ double sh[kMsBlock / 64];
    if (!st->any) return;
    const double a = st->a;
    const int64_t i0 = (int64_t)blockIdx.x * kMsSpan;
    const int64_t i1 = min(N, i0 + kMsSpan);
    double v = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kMsBlock) {
        const double ri = r[i] - a * q[i];
        r[i] = ri;
        v += ri * ri;
    }
    v = ms_block_sum(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// new r.r; b; every shift's zeta, a^s, b^s and convergence (one thread per
// shift); iteration count and the limits
__global__ __launch_bounds__(kMsBlock) void ms_shift_scal_kernel(MsShift *__restrict__ sh_tab,
                                                                 int S, MsState *__restrict__ st,
                                                                 const double *__restrict__ partial,
                                                                 int nblk) {
    __shared__ double sh[kMsBlock / 64];
    __shared__ int any_sh;
    __shared__ double rr_sh;
    if (!st->any) return;
    const double rr0 = ms_sum_partials(partial, nblk, sh);  // valid in thread 0
    if (threadIdx.x == 0) {
        any_sh = 0;
        rr_sh = rr0;
    }
    __syncthreads();
    const double rr = rr_sh;  // every shift's thread needs it
    const MsState t = *st;
    const double b = t.rr > 0.0 ? rr / t.rr : 0.0;
    const bool last = t.iters + 1 >= t.maxit;
    for (int s = threadIdx.x; s < S; s += kMsBlock) {
        MsShift e = sh_tab[s];
        e.upd = e.active;
        if (e.active) {
            const double den = t.a * t.b_prev * (e.zeta_prev - e.zeta) +
                               e.zeta_prev * t.a_prev * (1.0 + e.sigma * t.a);
            const double zn = e.zeta * e.zeta_prev * t.a_prev / den;
            const double ratio = zn / e.zeta;
            e.as = t.a * ratio;
            e.bs = ratio * ratio * b;
            e.zeta_prev = e.zeta;
            e.zeta = zn;
            e.res2 = zn * zn * rr;
            e.iters = t.iters + 1;
            if (!isfinite(zn) || !isfinite(rr)) {
                e.active = 0;
                e.upd = 0;
            } else if (e.res2 <= t.tol2 * t.ynorm2 || last) {
                e.active = 0;  // this iteration's x update is its last
            }
        }
        if (e.active) atomicOr(&any_sh, 1);
        sh_tab[s] = e;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        MsState u = t;
        u.apply = 1;
        u.iters = t.iters + 1;
        u.a_prev = t.a;
        u.b_prev = b;
        u.b = b;
        u.rr = rr;
        if (!isfinite(rr)) {
            u.any = 0;
            u.status = 2;
        } else if (!any_sh) {
            u.any = 0;
            u.status = last ? 3 : 1;
        }
        *st = u;
    }
}

// every updating shift: x^s += a^s p^s; every still active shift:
// p^s = zeta r + b^s p^s
__global__ __launch_bounds__(kMsBlock) void ms_update_kernel(const double *__restrict__ r,
                                                             const MsShift *__restrict__ sh_tab,
                                                             int S, int64_t N,
                                                             const MsState *__restrict__ st) {
    __shared__ MsShift tab[kMaxShifts];
    __shared__ int anyu;
    if (!st->apply) return;
    if (threadIdx.x == 0) anyu = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < S; s += kMsBlock) {
        tab[s] = sh_tab[s];
        if (tab[s].upd) atomicOr(&anyu, 1);
    }
    __syncthreads();
    if (!anyu) return;
    const int64_t i0 = (int64_t)blockIdx.x * kMsSpan;
    const int64_t i1 = min(N, i0 + kMsSpan);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kMsBlock) {
        const double ri = r[i];
        for (int s = 0; s < S; ++s) {
            const MsShift &e = tab[s];
            if (!e.upd) continue;
            const double pi = e.p[i];
            e.x[i] += e.as * pi;
            if (e.active) e.p[i] = e.zeta * ri + e.bs * pi;
        }
    }
}

// rs = y - q (q = (K~ + lambda_s I) x_s, column s of N x S), partial rs.rs
// per column (blocks: nblk per column)
__global__ __launch_bounds__(kMsBlock) void ms_resid_kernel(const double *__restrict__ y,
                                                            double *__restrict__ q, int64_t N,
                                                            int nblk, double *__restrict__ partial) {
    __shared__ double sh[kMsBlock / 64];
    const int s = blockIdx.x / nblk, lb = blockIdx.x % nblk;
    double *qs = q + (size_t)s * (size_t)N;
    const int64_t i0 = (int64_t)lb * kMsSpan;
    const int64_t i1 = min(N, i0 + kMsSpan);
    double v = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kMsBlock) {
        const double ri = y[i] - qs[i];
        qs[i] = ri;
        v += ri * ri;
    }
    v = ms_block_sum(v, sh);
    if (threadIdx.x == 0) partial[(size_t)s * nblk + lb] = v;
}

// out[s] = fixed-order sum of column s's partials (one workgroup per column)
__global__ __launch_bounds__(kMsBlock) void ms_col_sums_kernel(const double *__restrict__ partial,
                                                               int nblk, double *__restrict__ out) {
    __shared__ double sh[kMsBlock / 64];
    const double v = ms_sum_partials(partial + (size_t)blockIdx.x * nblk, nblk, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// A captured run of kCheckEvery iterations and the stream it was captured on.
struct MsGraph {
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    ~MsGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

// x += d
__global__ __launch_bounds__(kMsBlock) void ms_axpy_kernel(double *__restrict__ x,
                                                           const double *__restrict__ d, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * kMsBlock + threadIdx.x;
    if (i < N) x[i] += d[i];
}

}  // namespace

}  // namespace anova

using namespace anova;

extern "C" anova_status krr_cg_solve_shifts(anova_plan_t plan, const double *y, double *alpha,
                                            int32_t nshift, const double *shifts, int64_t ld,
                                            double tol, int32_t maxit, krr_cg_info *info,
                                            void *stream) {
    anova_status result = ANOVA_OK;
    const anova_status st = [&]() -> anova_status {
        try {
            ANOVA_REQUIRE(plan != nullptr, "NULL plan");
            ANOVA_REQUIRE(y != nullptr && alpha != nullptr && shifts != nullptr, "NULL argument");
            ANOVA_REQUIRE(nshift >= 1 && nshift <= kMaxShifts, "nshift must be in [1, 32]");
            ANOVA_REQUIRE(ld >= plan->N, "ld must be >= N");
            ANOVA_REQUIRE(std::isfinite(tol) && tol >= 0.0, "tol must be >= 0");
            ANOVA_REQUIRE(maxit >= 1, "maxit must be >= 1");
            for (int s = 0; s < nshift; ++s)
                ANOVA_REQUIRE(std::isfinite(shifts[s]) && shifts[s] > 0.0,
                              "every shift must be finite and > 0");
            hipStream_t s = (hipStream_t)stream;
            const int64_t N = plan->N;
            const int S = nshift;
            const int nblk = (int)((N + kMsSpan - 1) / kMsSpan);
            const double lam0 = *std::min_element(shifts, shifts + S);
            // shift 0 of the table is the base system (a smallest lambda)
            std::vector<int> order(S);
            for (int k = 0; k < S; ++k) order[k] = k;
            std::stable_sort(order.begin(), order.end(),
                             [&](int a, int b) { return shifts[a] < shifts[b]; });
            // work space: r, q, S directions (later S residual products and
            // right-hand sides), partials, scalars
            DevBuf work, tab, state, part, sums;
            const size_t vb = ((size_t)N * sizeof(double) + 255) & ~(size_t)255;
            work.alloc(vb * (2 + (size_t)S));
            char *wb = work.as<char>();
            double *r = reinterpret_cast<double *>(wb);
            double *q = reinterpret_cast<double *>(wb + vb);
            double *pbase = reinterpret_cast<double *>(wb + 2 * vb);
            std::vector<MsShift> htab(S);
            for (int k = 0; k < S; ++k) {
                MsShift e{};
                e.x = alpha + (size_t)order[k] * (size_t)ld;
                e.p = reinterpret_cast<double *>(wb + (2 + (size_t)k) * vb);
                e.sigma = shifts[order[k]] - lam0;
                htab[k] = e;
            }
            upload(tab, htab);
            state.alloc(sizeof(MsState));
            part.alloc((size_t)std::max(nblk, 1) * (size_t)S * sizeof(double));
            sums.alloc((size_t)S * sizeof(double));
            MsShift *dtab = tab.as<MsShift>();
            MsState *dst = state.as<MsState>();
            double *dpart = part.as<double>();
            // the base product q = (K~ + lambda_min I) p^0, batched like anova_matvec
            Batch prod;
            {
                BatchProblem bp;
                bp.plan = plan;
                bp.alpha = pbase;
                bp.out = q;
                bp.nrhs = 1;
                bp.ld = N;
                bp.beta = lam0;
                prod.build({bp});
            }
            // one iteration: the product, then five small kernels; the
            // launches after the last shift stops change nothing, so
            // kCheckEvery iterations are captured into one graph and the
            // host checks for completion between replays
            auto record = [&](hipStream_t cs) {
                prod.run(cs);
                hipLaunchKernelGGL(ms_dot_kernel, dim3(nblk), dim3(kMsBlock), 0, cs, pbase, q, N,
                                   dst, dpart);
                hipLaunchKernelGGL(ms_alpha_kernel, dim3(1), dim3(kMsBlock), 0, cs, dst, dpart,
                                   nblk);
                hipLaunchKernelGGL(ms_update_r_kernel, dim3(nblk), dim3(kMsBlock), 0, cs, r, q, N,
                                   dst, dpart);
                hipLaunchKernelGGL(ms_shift_scal_kernel, dim3(1), dim3(kMsBlock), 0, cs, dtab, S,
                                   dst, dpart, nblk);
                hipLaunchKernelGGL(ms_update_kernel, dim3(nblk), dim3(kMsBlock), 0, cs, r, dtab,
                                   S, N, dst);
                ANOVA_HIP_CHECK(hipGetLastError());
            };
            MsGraph G;
            {
                // capturing must not overlap other threads' allocations
                std::lock_guard<std::recursive_mutex> lock(device_mutex());
                ANOVA_HIP_CHECK(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
                hipGraph_t g = nullptr;
                ANOVA_HIP_CHECK(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
                try {
                    for (int j = 0; j < kCheckEvery; ++j) record(G.cap);
                } catch (...) {
                    (void)hipStreamEndCapture(G.cap, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                ANOVA_HIP_CHECK(hipStreamEndCapture(G.cap, &g));
                const hipError_t e = hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                ANOVA_HIP_CHECK(e);
            }
            hipLaunchKernelGGL(ms_init_kernel, dim3(nblk), dim3(kMsBlock), 0, s, y, r, dtab, S, N,
                               dpart);
            hipLaunchKernelGGL(ms_init_scal_kernel, dim3(1), dim3(kMsBlock), 0, s, dtab, S, dst,
                               dpart, nblk, tol, maxit);
            ANOVA_HIP_CHECK(hipGetLastError());
            MsState hst{};
            for (;;) {
                ANOVA_HIP_CHECK(hipMemcpyAsync(&hst, dst, sizeof(MsState), hipMemcpyDeviceToHost,
                                               s));
                ANOVA_HIP_CHECK(hipStreamSynchronize(s));
                if (!hst.any) break;
                ANOVA_HIP_CHECK(hipGraphLaunch(G.exec, s));
            }
            std::vector<MsShift> fin(S);
            ANOVA_HIP_CHECK(hipMemcpyAsync(fin.data(), dtab, (size_t)S * sizeof(MsShift),
                                           hipMemcpyDeviceToHost, s));
            ANOVA_HIP_CHECK(hipStreamSynchronize(s));
            if (hst.status == 2) throw Error{ANOVA_E_BREAKDOWN, "CG breakdown (p^T A p <= 0 or NaN)"};
            // true residuals y - (K~ + lambda_s I) x_s with the float64
            // product, into the direction slots (N x S)
            double *qs = pbase;
            {
                std::vector<BatchProblem> bps((size_t)S);
                for (int k = 0; k < S; ++k) {
                    BatchProblem &bp = bps[(size_t)k];
                    bp.plan = plan;
                    bp.alpha = htab[k].x;
                    bp.out = qs + (size_t)k * (size_t)N;
                    bp.nrhs = 1;
                    bp.ld = N;
                    bp.beta = shifts[order[k]];
                    bp.residual = true;
                }
                Batch rb;
                rb.build(bps);
                rb.run(s);
                hipLaunchKernelGGL(ms_resid_kernel, dim3(nblk * S), dim3(kMsBlock), 0, s, y, qs, N,
                                   nblk, dpart);
                hipLaunchKernelGGL(ms_col_sums_kernel, dim3(S), dim3(kMsBlock), 0, s, dpart, nblk,
                                   sums.as<double>());
                ANOVA_HIP_CHECK(hipGetLastError());
                ANOVA_HIP_CHECK(hipStreamSynchronize(s));  // rb's work space dies here
            }
            std::vector<double> res2(S);
            ANOVA_HIP_CHECK(hipMemcpy(res2.data(), sums.ptr, (size_t)S * sizeof(double),
                                      hipMemcpyDeviceToHost));
            const double ynorm = std::sqrt(hst.ynorm2);
            std::vector<krr_cg_info> out(S);
            for (int k = 0; k < S; ++k) {
                krr_cg_info &inf = out[(size_t)order[k]];
                const double rn = std::sqrt(res2[(size_t)k]);
                inf.iters = fin[k].iters;
                inf.relres = ynorm > 0 ? std::sqrt(std::max(fin[k].res2, 0.0)) / ynorm : 0.0;
                inf.true_relres = ynorm > 0 ? rn / ynorm : 0.0;
                inf.converged = ynorm == 0.0 || rn <= tol * ynorm ? 1 : 0;
                if (inf.converged || hst.status == 2) continue;
                // refinement: (K~ + lambda_s I) d = r_s to tol ||y||, x_s += d
                const int left = std::max(1, maxit - hst.iters);
                krr_cg_info sub{};
                const anova_status cs =
                    krr_cg_solve(plan, qs + (size_t)k * (size_t)N, q, 1, N, shifts[order[k]],
                                 tol * ynorm / rn, left, &sub, stream);
                if (cs != ANOVA_OK && cs != ANOVA_E_NOT_CONVERGED)
                    throw Error{cs, get_error()};
                hipLaunchKernelGGL(ms_axpy_kernel, dim3((unsigned)((N + kMsBlock - 1) / kMsBlock)),
                                   dim3(kMsBlock), 0, s, htab[k].x, q, N);
                ANOVA_HIP_CHECK(hipGetLastError());
                inf.iters += sub.iters;
                inf.true_relres = sub.true_relres * rn / ynorm;
                inf.relres = sub.relres * rn / ynorm;
                inf.converged = sub.converged;
            }
            ANOVA_HIP_CHECK(hipStreamSynchronize(s));
            bool all = true;
            for (const krr_cg_info &inf : out) all = all && inf.converged;
            if (info)
                for (int k = 0; k < S; ++k) info[k] = out[(size_t)k];
            result = all ? ANOVA_OK : ANOVA_E_NOT_CONVERGED;
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
    }();
    if (st != ANOVA_OK) return st;
    if (result == ANOVA_E_NOT_CONVERGED) set_error("some shift reached maxit");
    return result;
}
