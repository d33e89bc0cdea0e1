// Conjugate gradients for (K~ + beta I) alpha = y (Sec. 2: the system is
// symmetric positive definite for beta > 0 and is solved by CG with one
// kernel product per iteration; no preconditioner, Sec. 6).
//
// Everything except the kernel product runs in float64 on the device: dot
// products are two-stage reductions (per-block partial sums, then one
// workgroup per column adding the partials in a fixed order, so results do
// not depend on scheduling), and the CG scalars stay in device memory, so an
// iteration needs no host round trip.  Each iteration is captured once into a
// hipGraph and replayed; the host reads the convergence flags every few
// iterations.  Every kResidualPeriod iterations the recursive residual is
// replaced by y - A x (residual replacement), and at exit the true residual
// is recomputed for the report.
#include <algorithm>
#include <cmath>

#include "anova_internal.h"

namespace anova {

constexpr int kRedBlock = 256;
constexpr int kResidualPeriod = 50;
constexpr int kCheckEvery = 8;

struct CgScal {
    double rho;      // r.r of the current residual
    double ynorm2;   // y.y
    double tol2;     // tol^2
    double a, b;     // step length and direction update
    double pq;       // p.q of the current iteration
    int32_t active;  // 1 while the column iterates
    int32_t status;  // 0 running/converged, 1 converged, 2 breakdown
    int32_t iters;
    int32_t pad;
};

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    }
    __syncthreads();
    return t;  // valid in thread 0
}

// partial[c*nblk + blockIdx.x] = sum over this block's share of a_c . b_c
__global__ __launch_bounds__(kRedBlock) void dot_partial_kernel(
    const double *__restrict__ a, int64_t lda, const double *__restrict__ b, int64_t ldb,
    int64_t N, double *__restrict__ partial, int nblk) {
    __shared__ double sh[kRedBlock / 64];
    const int c = blockIdx.y;
    const double *ac = a + (size_t)c * lda;
    const double *bc = b + (size_t)c * ldb;
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; i < N;
         i += (int64_t)nblk * kRedBlock)
        v += ac[i] * bc[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) partial[(size_t)c * nblk + blockIdx.x] = v;
}

__device__ double sum_partials(const double *__restrict__ partial, int nblk, double *sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += kRedBlock) v += partial[i];
    return block_sum(v, sh);
}

// ---------------------------------------------------------------- CG steps
// x = 0, r = y, p = y, partial r.r
__global__ __launch_bounds__(kRedBlock) void cg_init_kernel(
    const double *__restrict__ y, int64_t ldy, double *__restrict__ x, int64_t ldx,
    double *__restrict__ r, double *__restrict__ p, int64_t N, double *__restrict__ partial,
    int nblk) {
    __shared__ double sh[kRedBlock / 64];
    const int c = blockIdx.y;
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; i < N;
         i += (int64_t)nblk * kRedBlock) {
        const double yi = y[(size_t)c * ldy + i];
        x[(size_t)c * ldx + i] = 0.0;
        r[(size_t)c * N + i] = yi;
        p[(size_t)c * N + i] = yi;
        v += yi * yi;
    }
    v = block_sum(v, sh);
    if (threadIdx.x == 0) partial[(size_t)c * nblk + blockIdx.x] = v;
}

__global__ __launch_bounds__(kRedBlock) void cg_init_scal_kernel(
    const double *__restrict__ partial, int nblk, CgScal *__restrict__ sc, double tol) {
    __shared__ double sh[kRedBlock / 64];
    const int c = blockIdx.x;
    const double y2 = sum_partials(partial + (size_t)c * nblk, nblk, sh);
    if (threadIdx.x == 0) {
        CgScal s{};
        s.rho = y2;
        s.ynorm2 = y2;
        s.tol2 = tol * tol;
        s.active = (y2 > 0.0 && std::isfinite(y2)) ? 1 : 0;
        s.status = y2 > 0.0 ? (std::isfinite(y2) ? 0 : 2) : 1;
        s.iters = 0;
        sc[c] = s;
    }
}

// a = rho / (p.q)
__global__ __launch_bounds__(kRedBlock) void cg_alpha_kernel(
    const double *__restrict__ partial, int nblk, CgScal *__restrict__ sc) {
    __shared__ double sh[kRedBlock / 64];
    const int c = blockIdx.x;
    const double pq = sum_partials(partial + (size_t)c * nblk, nblk, sh);
    if (threadIdx.x == 0) {
        CgScal s = sc[c];
        s.pq = pq;
        if (s.active) {
            if (!(pq > 0.0) || !std::isfinite(pq)) {
                s.active = 0;
                s.status = 2;
            } else {
                s.a = s.rho / pq;
            }
        }
        sc[c] = s;
    }
}

// x += a p; r -= a q; partial r.r
__global__ __launch_bounds__(kRedBlock) void cg_update_xr_kernel(
    double *__restrict__ x, int64_t ldx, double *__restrict__ r, const double *__restrict__ p,
    const double *__restrict__ q, int64_t N, const CgScal *__restrict__ sc,
    double *__restrict__ partial, int nblk) {
    __shared__ double sh[kRedBlock / 64];
    const int c = blockIdx.y;
    const bool act = sc[c].active != 0;
    const double a = sc[c].a;
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; i < N;
         i += (int64_t)nblk * kRedBlock) {
        double ri = r[(size_t)c * N + i];
        if (act) {
            x[(size_t)c * ldx + i] += a * p[(size_t)c * N + i];
            ri -= a * q[(size_t)c * N + i];
            r[(size_t)c * N + i] = ri;
        }
        v += ri * ri;
    }
    v = block_sum(v, sh);
    if (threadIdx.x == 0) partial[(size_t)c * nblk + blockIdx.x] = v;
}

// r = y - q (q = A x); partial r.r
__global__ __launch_bounds__(kRedBlock) void cg_replace_kernel(
    const double *__restrict__ y, int64_t ldy, double *__restrict__ r,
    const double *__restrict__ q, int64_t N, const CgScal *__restrict__ sc,
    double *__restrict__ partial, int nblk, int force) {
    __shared__ double sh[kRedBlock / 64];
    const int c = blockIdx.y;
    const bool act = force || sc[c].active != 0;
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; i < N;
         i += (int64_t)nblk * kRedBlock) {
        double ri;
        if (act) {
            ri = y[(size_t)c * ldy + i] - q[(size_t)c * N + i];
            r[(size_t)c * N + i] = ri;
        } else {
            ri = r[(size_t)c * N + i];
        }
        v += ri * ri;
    }
    v = block_sum(v, sh);
    if (threadIdx.x == 0) partial[(size_t)c * nblk + blockIdx.x] = v;
}

// rho' = r.r; convergence test; b = rho'/rho
__global__ __launch_bounds__(kRedBlock) void cg_beta_kernel(
    const double *__restrict__ partial, int nblk, CgScal *__restrict__ sc) {
    __shared__ double sh[kRedBlock / 64];
    const int c = blockIdx.x;
    const double rr = sum_partials(partial + (size_t)c * nblk, nblk, sh);
    if (threadIdx.x == 0) {
        CgScal s = sc[c];
        if (s.active) {
            s.iters += 1;
            if (!std::isfinite(rr)) {
                s.active = 0;
                s.status = 2;
            } else if (rr <= s.tol2 * s.ynorm2) {
                s.active = 0;
                s.status = 1;
                s.rho = rr;
            } else {
                s.b = rr / s.rho;
                s.rho = rr;
            }
        }
        sc[c] = s;
    }
}

// p = r + b p
__global__ __launch_bounds__(kRedBlock) void cg_update_p_kernel(
    double *__restrict__ p, const double *__restrict__ r, int64_t N,
    const CgScal *__restrict__ sc, int nblk) {
    const int c = blockIdx.y;
    if (!sc[c].active) return;
    const double b = sc[c].b;
    for (int64_t i = blockIdx.x * (int64_t)kRedBlock + threadIdx.x; i < N;
         i += (int64_t)nblk * kRedBlock)
        p[(size_t)c * N + i] = r[(size_t)c * N + i] + b * p[(size_t)c * N + i];
}

// ---------------------------------------------------------------- solver
struct Solver {
    anova_plan_s *plan = nullptr;
    int nrhs = 0;
    int64_t N = 0;
    int nblk = 0;
    DevBuf r, p, q, partial, scal;
    hipStream_t cap = nullptr;
    hipGraphExec_t g_plain = nullptr, g_replace = nullptr;
    ~Solver() {
        if (g_plain) (void)hipGraphExecDestroy(g_plain);
        if (g_replace) (void)hipGraphExecDestroy(g_replace);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

static void apply_A(Solver &S, const double *x, int64_t ldx, double *y, double beta,
                    hipStream_t s) {
    for (int c = 0; c < S.nrhs; ++c)
        plan_matvec(S.plan, x + (size_t)c * ldx, y + (size_t)c * S.N, beta, s);
}

static void record_iteration(Solver &S, double *x, int64_t ldx, const double *y, int64_t ldy,
                             double beta, bool replace, hipStream_t s) {
    const dim3 g2(S.nblk, S.nrhs);
    double *r = S.r.as<double>(), *p = S.p.as<double>(), *q = S.q.as<double>();
    double *part = S.partial.as<double>();
    CgScal *sc = S.scal.as<CgScal>();
    apply_A(S, p, S.N, q, beta, s);
    hipLaunchKernelGGL(dot_partial_kernel, g2, dim3(kRedBlock), 0, s, p, S.N, q, S.N, S.N, part,
                       S.nblk);
    hipLaunchKernelGGL(cg_alpha_kernel, dim3(S.nrhs), dim3(kRedBlock), 0, s, part, S.nblk, sc);
    hipLaunchKernelGGL(cg_update_xr_kernel, g2, dim3(kRedBlock), 0, s, x, ldx, r, p, q, S.N, sc,
                       part, S.nblk);
    if (replace) {
        apply_A(S, x, ldx, q, beta, s);
        hipLaunchKernelGGL(cg_replace_kernel, g2, dim3(kRedBlock), 0, s, y, ldy, r, q, S.N, sc,
                           part, S.nblk, 0);
    }
    hipLaunchKernelGGL(cg_beta_kernel, dim3(S.nrhs), dim3(kRedBlock), 0, s, part, S.nblk, sc);
    hipLaunchKernelGGL(cg_update_p_kernel, g2, dim3(kRedBlock), 0, s, p, r, S.N, sc, S.nblk);
    ANOVA_HIP_CHECK(hipGetLastError());
}

static hipGraphExec_t capture(Solver &S, double *x, int64_t ldx, const double *y, int64_t ldy,
                              double beta, bool replace) {
    hipGraph_t g = nullptr;
    // per-stage event timing is not recorded inside graphs
    const bool timing = S.plan->timing;
    S.plan->timing = false;
    ANOVA_HIP_CHECK(hipStreamBeginCapture(S.cap, hipStreamCaptureModeThreadLocal));
    try {
        record_iteration(S, x, ldx, y, ldy, beta, replace, S.cap);
    } catch (...) {
        (void)hipStreamEndCapture(S.cap, &g);
        if (g) (void)hipGraphDestroy(g);
        S.plan->timing = timing;
        throw;
    }
    S.plan->timing = timing;
    ANOVA_HIP_CHECK(hipStreamEndCapture(S.cap, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    ANOVA_HIP_CHECK(e);
    return ex;
}

}  // namespace anova

using namespace anova;

extern "C" anova_status krr_cg_solve(anova_plan_t plan, const double *y, double *alpha,
                                     int32_t nrhs, int64_t ld, double beta, double tol,
                                     int32_t maxit, krr_cg_info *info, void *stream) {
    anova_status result = ANOVA_OK;
    try {
        ANOVA_REQUIRE(plan != nullptr, "NULL plan");
        ANOVA_REQUIRE(y != nullptr && alpha != nullptr, "NULL vector");
        ANOVA_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        ANOVA_REQUIRE(ld >= plan->N, "ld must be >= N");
        ANOVA_REQUIRE(std::isfinite(beta) && beta > 0, "beta must be finite and > 0");
        ANOVA_REQUIRE(std::isfinite(tol) && tol >= 0, "tol must be finite and >= 0");
        ANOVA_REQUIRE(maxit >= 1, "maxit must be >= 1");
        hipStream_t s = (hipStream_t)stream;
        Solver S;
        S.plan = plan;
        S.nrhs = nrhs;
        S.N = plan->N;
        S.nblk = (int)std::min<int64_t>((S.N + 4 * kRedBlock - 1) / (4 * kRedBlock), 1024);
        const size_t vec = (size_t)S.N * nrhs * sizeof(double);
        S.r.alloc(vec);
        S.p.alloc(vec);
        S.q.alloc(vec);
        S.partial.alloc((size_t)S.nblk * nrhs * sizeof(double));
        S.scal.alloc(sizeof(CgScal) * nrhs);
        ensure_grid(plan, 1);
        ANOVA_HIP_CHECK(hipStreamCreateWithFlags(&S.cap, hipStreamNonBlocking));
        const dim3 g2(S.nblk, nrhs);
        hipLaunchKernelGGL(cg_init_kernel, g2, dim3(kRedBlock), 0, s, y, ld, alpha, ld,
                           S.r.as<double>(), S.p.as<double>(), S.N, S.partial.as<double>(),
                           S.nblk);
        hipLaunchKernelGGL(cg_init_scal_kernel, dim3(nrhs), dim3(kRedBlock), 0, s,
                           S.partial.as<double>(), S.nblk, S.scal.as<CgScal>(), tol);
        ANOVA_HIP_CHECK(hipGetLastError());
        S.g_plain = capture(S, alpha, ld, y, ld, beta, false);
        S.g_replace = capture(S, alpha, ld, y, ld, beta, true);
        std::vector<CgScal> hs(nrhs);
        int it = 0;
        ANOVA_HIP_CHECK(hipMemcpyAsync(hs.data(), S.scal.ptr, sizeof(CgScal) * nrhs,
                                       hipMemcpyDeviceToHost, s));
        ANOVA_HIP_CHECK(hipStreamSynchronize(s));
        auto any_active = [&] {
            for (auto &c : hs)
                if (c.active) return true;
            return false;
        };
        while (it < maxit && any_active()) {
            const int k = std::min(kCheckEvery, maxit - it);
            for (int j = 0; j < k; ++j) {
                const bool rep = ((it + j + 1) % kResidualPeriod) == 0;
                ANOVA_HIP_CHECK(hipGraphLaunch(rep ? S.g_replace : S.g_plain, s));
            }
            it += k;
            ANOVA_HIP_CHECK(hipMemcpyAsync(hs.data(), S.scal.ptr, sizeof(CgScal) * nrhs,
                                           hipMemcpyDeviceToHost, s));
            ANOVA_HIP_CHECK(hipStreamSynchronize(s));
        }
        // true residual at exit: r = y - A x (all columns)
        apply_A(S, alpha, ld, S.q.as<double>(), beta, s);
        hipLaunchKernelGGL(cg_replace_kernel, g2, dim3(kRedBlock), 0, s, y, ld, S.r.as<double>(),
                           S.q.as<double>(), S.N, S.scal.as<CgScal>(), S.partial.as<double>(),
                           S.nblk, 1);
        ANOVA_HIP_CHECK(hipGetLastError());
        std::vector<double> part((size_t)S.nblk * nrhs);
        ANOVA_HIP_CHECK(hipMemcpyAsync(part.data(), S.partial.ptr, part.size() * sizeof(double),
                                       hipMemcpyDeviceToHost, s));
        ANOVA_HIP_CHECK(hipMemcpyAsync(hs.data(), S.scal.ptr, sizeof(CgScal) * nrhs,
                                       hipMemcpyDeviceToHost, s));
        ANOVA_HIP_CHECK(hipStreamSynchronize(s));
        bool all_conv = true, breakdown = false;
        for (int c = 0; c < nrhs; ++c) {
            double tr = 0.0;
            for (int b = 0; b < S.nblk; ++b) tr += part[(size_t)c * S.nblk + b];
            const CgScal &sc = hs[c];
            const bool conv = sc.status == 1;
            all_conv = all_conv && conv;
            breakdown = breakdown || sc.status == 2;
            if (info) {
                info[c].iters = sc.iters;
                info[c].converged = conv ? 1 : 0;
                info[c].relres = sc.ynorm2 > 0 ? std::sqrt(sc.rho / sc.ynorm2) : 0.0;
                info[c].true_relres = sc.ynorm2 > 0 ? std::sqrt(tr / sc.ynorm2) : 0.0;
            }
        }
        if (breakdown) {
            set_error("CG breakdown (p^T A p <= 0 or a non-finite value)");
            result = ANOVA_E_BREAKDOWN;
        } else if (!all_conv) {
            set_error("CG reached maxit before the tolerance");
            result = ANOVA_E_NOT_CONVERGED;
        }
    } catch (const Error &e) {
        set_error(e.msg);
        return e.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return ANOVA_E_NOMEM;
    }
    return result;
}
