// Hot-path kernels of one window's fast summation (gfx950, wave64):
//   spread   : first step of the adjoint NFFT (Sec. 4.1, eq. adjnfft) --
//              point coefficients are spread onto the oversampled grid with a
//              compactly supported window, accumulated per grid tile in LDS;
//   convolve : d_A-dimensional FFT, multiplication by the kernel's Fourier
//              coefficients over the window transform squared, inverse FFT
//              (Sec. 4.2, eq. fastsum); the multiplier is a product over
//              dimensions, so the three steps factor into one
//              forward-FFT / multiply / inverse-FFT pass per axis;
//   gather   : last step of the NFFT (Sec. 4.1, eq. nfft) -- the grid is
//              interpolated back at the points with the same window, weighted
//              by eta_l and accumulated in float64 (Sec. 5, K = sum eta_l K_l).
//
// Points are sorted by grid tile at plan time.  A work item ("sub-problem")
// is a run of points of one tile; its workgroup owns the tile plus a halo of
// 2m-1 grid points in LDS, accumulates there with integer LDS atomics and
// stores the finished region to a private buffer; a fold kernel then adds
// the overlapping regions into the grid in a fixed order.  Every step is
// deterministic, so a matvec gives bitwise identical results run to run.
#include "anova_internal.h"

namespace anova {

template <typename T> struct NodeOf;
template <> struct NodeOf<float> { using type = NodeF32; };
template <> struct NodeOf<double> { using type = NodeF64; };
template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

constexpr int kBlock = 256;

// Weights phi0(f + m - 1 - a), a = 0..W-1, of a point with fractional cell
// offset f in [0,1): one polynomial per support offset, Horner in z = 2f-1.
template <typename T, int W>
__device__ __forceinline__ void window_weights(const T *__restrict__ poly, int deg, T f,
                                               T (&w)[W]) {
    const T z = T(2) * f - T(1);
#pragma unroll
    for (int a = 0; a < W; ++a) w[a] = poly[a * (deg + 1) + deg];
    for (int k = deg - 1; k >= 0; --k) {
#pragma unroll
        for (int a = 0; a < W; ++a) w[a] = w[a] * z + poly[a * (deg + 1) + k];
    }
}

__device__ __forceinline__ int wrap_index(int g, int n) {
    g %= n;
    return g < 0 ? g + n : g;
}

// ------------------------------------------------------------------ spread
// Fixed-point accumulation.  LDS float atomics are slow on this chip while
// 64-bit integer LDS atomics run at full rate, and integer sums are exact, so
// each workgroup accumulates its tile region in int64: a contribution v is
// rounded to an integer at the workgroup's scale 2^S, chosen from the largest
// |alpha| of its points so that no contribution exceeds 2^30 (float32 path,
// rounding 2^-31 of max|alpha|) or 2^52 (float64 path) in magnitude; the sum
// of at most 1024 such terms cannot overflow.  The result does not depend on
// the order of the atomic additions.
__device__ __forceinline__ long long round_to_ll(float x) {  // |x| < 2^31
    return (long long)__float2int_rn(x);
}
__device__ __forceinline__ long long round_to_ll(double x) {  // |x| < 2^62
    x = rint(x);
    const double hi = floor(x * 0x1p-32);       // exact: |hi| < 2^30
    const double lo = x - hi * 0x1p32;          // exact, in [0, 2^32)
    return (long long)((unsigned long long)(long long)(int)hi << 32) + (long long)(unsigned)lo;
}
template <typename T> struct FixedBits;
template <> struct FixedBits<float> { static constexpr int value = 30; };
template <> struct FixedBits<double> { static constexpr int value = 52; };

__device__ __forceinline__ float block_max(float v, float *sh) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    float r = sh[0];
    for (int i = 1; i < kBlock / 64; ++i) r = fmaxf(r, sh[i]);
    __syncthreads();
    return r;
}

// One workgroup per sub-problem: spreads its points into the LDS image of
// its tile plus halo and stores that region (as T) to its private slice of
// `priv`; the fold kernel adds the regions into the grid.
template <typename T, int DA, int W>
__global__ __launch_bounds__(kBlock) void spread_kernel(
    const typename NodeOf<T>::type *__restrict__ nodes, const int32_t *__restrict__ perm,
    const SubProblem *__restrict__ subs, const double *__restrict__ alpha, T *__restrict__ priv,
    const T *__restrict__ poly, int deg, int tile, int tpd) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem_raw);
    __shared__ float red[kBlock / 64];
    const int L = tile + W - 1;
    const int L2 = DA >= 2 ? L * L : L;
    const int vol = DA == 3 ? L2 * L : L2;
    for (int e = threadIdx.x; e < vol; e += kBlock) acc[e] = 0ull;
    const SubProblem sp = subs[blockIdx.x];
    const int end = sp.start + sp.count;
    float amax = 0.0f;
    for (int j = sp.start + threadIdx.x; j < end; j += kBlock) {
        float va = (float)fabs(alpha[perm[j]]);
        if (!(va <= 3.0e38f)) va = INFINITY;  // NaN or out of range: propagate as NaN below
        amax = fmaxf(amax, va);
    }
    amax = block_max(amax, red);  // also orders the zero fill before the adds
    T *out = priv + (size_t)blockIdx.x * vol;
    if (!(amax > 0.0f) || !isfinite(amax)) {
        // all-zero (or non-finite) coefficients: the region is zero (or NaN)
        const T fill = amax > 0.0f ? T(NAN) : T(0);
        for (int e = threadIdx.x; e < vol; e += kBlock) out[e] = fill;
        return;
    }
    int ex2;
    (void)frexpf(amax * 1.0000002f, &ex2);  // amax * (1 + margin) < 2^ex2
    const int S = FixedBits<T>::value - ex2;
    const T sc = (T)ldexp(1.0, S);
    const int ox = (sp.tile % tpd) * tile;
    const int oy = ((sp.tile / tpd) % tpd) * tile;
    const int oz = (sp.tile / (tpd * tpd)) * tile;
    for (int j = sp.start + threadIdx.x; j < end; j += kBlock) {
        const auto rec = nodes[j];
        const T a = static_cast<T>(alpha[perm[j]]) * sc;
        const int lx = int(rec.cell & 1023u) - ox;
        T wx[W];
        window_weights<T, W>(poly, deg, rec.f[0], wx);
        if constexpr (DA == 1) {
#pragma unroll
            for (int i = 0; i < W; ++i)
                atomicAdd(&acc[lx + i], (unsigned long long)round_to_ll(a * wx[i]));
        } else {
            const int ly = int((rec.cell >> 10) & 1023u) - oy;
            T wy[W];
            window_weights<T, W>(poly, deg, rec.f[1], wy);
            if constexpr (DA == 2) {
#pragma unroll
                for (int b = 0; b < W; ++b) {
                    const T wb = a * wy[b];
                    unsigned long long *row = acc + (ly + b) * L + lx;
#pragma unroll
                    for (int i = 0; i < W; ++i)
                        atomicAdd(&row[i], (unsigned long long)round_to_ll(wb * wx[i]));
                }
            } else {
                const int lz = int(rec.cell >> 20) - oz;
                T wz[W];
                window_weights<T, W>(poly, deg, rec.f[2], wz);
                for (int c = 0; c < W; ++c) {
                    const T wc = a * wz[c];
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        const T wbc = wc * wy[b];
                        unsigned long long *row = acc + ((lz + c) * L + ly + b) * L + lx;
#pragma unroll
                        for (int i = 0; i < W; ++i)
                            atomicAdd(&row[i], (unsigned long long)round_to_ll(wbc * wx[i]));
                    }
                }
            }
        }
    }
    __syncthreads();
    const double inv = ldexp(1.0, -S);
    for (int e = threadIdx.x; e < vol; e += kBlock)
        out[e] = static_cast<T>((double)(long long)acc[e] * inv);
}

// ------------------------------------------------------------------ tile sum
// When a tile's points are split over several sub-problems, their regions
// are first added elementwise, in sub-problem order, into one region per
// non-empty tile: src_sub[k] .. src_sub[k+1]-1 are the sub-problems of the
// k-th non-empty tile.
template <typename T>
__global__ __launch_bounds__(kBlock) void tile_sum_kernel(
    const T *__restrict__ priv, const int32_t *__restrict__ src_sub, T *__restrict__ treg,
    int vol) {
    const int k = blockIdx.y;
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= vol) return;
    const int s0 = src_sub[k], s1 = src_sub[k + 1];
    double s = 0.0;
    for (int q = s0; q < s1; ++q) s += (double)priv[(size_t)q * vol + e];
    treg[(size_t)k * vol + e] = static_cast<T>(s);
}

// ------------------------------------------------------------------ fold
// One workgroup per destination tile: every grid point of the tile is the
// sum, in the fixed order of the plan's pair list, of the region values of
// all sub-problems whose region covers it (regions wrap periodically: per
// dimension the region indices of grid point o + c are the values in [0, L)
// congruent to b + c mod n, b the tile origin's offset in the region).
// Writes every grid point, so no zero fill is needed.
template <typename T, int DA>
__global__ __launch_bounds__(kBlock) void fold_kernel(
    const T *__restrict__ priv, const int2 *__restrict__ pairs,
    const int32_t *__restrict__ pair_start, T *__restrict__ grid, int n, int tile, int tpd,
    int L) {
    const int d = blockIdx.x;
    const int ox = (d % tpd) * tile;
    const int oy = ((d / tpd) % tpd) * tile;
    const int oz = (d / (tpd * tpd)) * tile;
    const int L2 = DA >= 2 ? L * L : L;
    const int vol = DA == 3 ? L2 * L : L2;
    int cells = tile;
    if (DA >= 2) cells *= tile;
    if (DA == 3) cells *= tile;
    const int p0 = pair_start[d], p1 = pair_start[d + 1];
    for (int c = threadIdx.x; c < cells; c += kBlock) {
        const int cx = c % tile;
        const int cy = DA >= 2 ? (c / tile) % tile : 0;
        const int cz = DA == 3 ? c / (tile * tile) : 0;
        double s = 0.0;
        for (int p = p0; p < p1; ++p) {
            const int2 pr = pairs[p];
            const T *reg = priv + (size_t)pr.x * vol;
            const int bx = pr.y & 1023, by = (pr.y >> 10) & 1023, bz = (pr.y >> 20) & 1023;
            // region indices congruent to the grid point mod n: the smallest
            // is (b + c) mod n, the others follow in steps of n while < L
            const int ex0 = (bx + cx) % n;
            const int ey0 = DA >= 2 ? (by + cy) % n : 0;
            const int ez0 = DA == 3 ? (bz + cz) % n : 0;
            for (int ez = ez0; ez < (DA == 3 ? L : 1); ez += n)
                for (int ey = ey0; ey < (DA >= 2 ? L : 1); ey += n)
                    for (int ex = ex0; ex < L; ex += n)
                        s += (double)reg[ez * L2 + ey * L + ex];
        }
        size_t g = (size_t)(ox + cx);
        if (DA >= 2) g += (size_t)n * (size_t)(oy + cy);
        if (DA == 3) g += (size_t)n * (size_t)n * (size_t)(oz + cz);
        grid[g] = static_cast<T>(s);
    }
}

// ------------------------------------------------------------------ gather
template <typename T, int DA, int W, bool FIRST>
__global__ __launch_bounds__(kBlock) void gather_kernel(
    const typename NodeOf<T>::type *__restrict__ nodes, const int32_t *__restrict__ perm,
    const SubProblem *__restrict__ subs, const T *__restrict__ grid,
    const double *__restrict__ alpha, double *__restrict__ out, double eta, double beta,
    const T *__restrict__ poly, int deg, int n, int tile, int tpd) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    constexpr int m = W / 2;
    const int L = tile + W - 1;
    const int L2 = DA >= 2 ? L * L : L;
    const int vol = DA == 3 ? L2 * L : L2;
    const SubProblem sp = subs[blockIdx.x];
    const int ox = (sp.tile % tpd) * tile;
    const int oy = ((sp.tile / tpd) % tpd) * tile;
    const int oz = (sp.tile / (tpd * tpd)) * tile;
    for (int e = threadIdx.x; e < vol; e += kBlock) {
        const int ex = e % L;
        size_t g = (size_t)wrap_index(ox - m + 1 + ex, n);
        if constexpr (DA >= 2) {
            const int ey = (e / L) % L;
            g += (size_t)n * (size_t)wrap_index(oy - m + 1 + ey, n);
        }
        if constexpr (DA == 3) {
            const int ez = e / L2;
            g += (size_t)n * (size_t)n * (size_t)wrap_index(oz - m + 1 + ez, n);
        }
        lds[e] = grid[g];
    }
    __syncthreads();
    const int end = sp.start + sp.count;
    for (int j = sp.start + threadIdx.x; j < end; j += kBlock) {
        const auto rec = nodes[j];
        const int lx = int(rec.cell & 1023u) - ox;
        T wx[W];
        window_weights<T, W>(poly, deg, rec.f[0], wx);
        T acc = T(0);
        if constexpr (DA == 1) {
#pragma unroll
            for (int i = 0; i < W; ++i) acc += lds[lx + i] * wx[i];
        } else {
            const int ly = int((rec.cell >> 10) & 1023u) - oy;
            T wy[W];
            window_weights<T, W>(poly, deg, rec.f[1], wy);
            if constexpr (DA == 2) {
#pragma unroll
                for (int b = 0; b < W; ++b) {
                    const T *row = lds + (ly + b) * L + lx;
                    T s = T(0);
#pragma unroll
                    for (int i = 0; i < W; ++i) s += row[i] * wx[i];
                    acc += s * wy[b];
                }
            } else {
                const int lz = int(rec.cell >> 20) - oz;
                T wz[W];
                window_weights<T, W>(poly, deg, rec.f[2], wz);
                for (int c = 0; c < W; ++c) {
                    T sc = T(0);
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        const T *row = lds + ((lz + c) * L + ly + b) * L + lx;
                        T s = T(0);
#pragma unroll
                        for (int i = 0; i < W; ++i) s += row[i] * wx[i];
                        sc += s * wy[b];
                    }
                    acc += sc * wz[c];
                }
            }
        }
        const int i = perm[j];
        const double v = eta * static_cast<double>(acc);
        if constexpr (FIRST)
            out[i] = beta * alpha[i] + v;
        else
            out[i] += v;
    }
}

// ------------------------------------------------------------------ convolve
// One pass along axis `ax` (element stride s = n^ax) of the n^d_A real grid:
// two real lines form one complex line; radix-2 Stockham FFT in LDS,
// multiplication by the real, even per-axis multiplier, inverse FFT.
// Because the multiplier is real and even, filtering x + i y equals
// filtering x and y separately.
template <typename T, int LOGN>
__global__ __launch_bounds__(kBlock) void convolve_kernel(
    T *__restrict__ grid, const T *__restrict__ bconv,
    const typename Cplx<T>::type *__restrict__ tw, int nlines, int s, int NP) {
    using C = typename Cplx<T>::type;
    constexpr int n = 1 << LOGN;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *bufA = reinterpret_cast<C *>(smem_raw);
    C *bufB = bufA + NP * n;
    const int q0 = blockIdx.x * NP;
    const bool contiguous = (s == 1);
    auto base_of = [&](int r) -> size_t {
        const size_t hi = (size_t)(r / s), lo = (size_t)(r % s);
        return hi * (size_t)s * n + lo;
    };
    for (int e = threadIdx.x; e < NP * n; e += kBlock) {
        int ql, u;
        if (contiguous) { ql = e / n; u = e % n; } else { u = e / NP; ql = e % NP; }
        const int r0 = 2 * (q0 + ql), r1 = r0 + 1;
        C v;
        v.x = r0 < nlines ? grid[base_of(r0) + (size_t)u * s] : T(0);
        v.y = r1 < nlines ? grid[base_of(r1) + (size_t)u * s] : T(0);
        bufA[ql * n + u] = v;
    }
    __syncthreads();
    C *src = bufA, *dst = bufB;
    // forward transform, X_k = sum_u x_u exp(-2 pi i k u / n)
    for (int Ns = 1; Ns < n; Ns <<= 1) {
        for (int e = threadIdx.x; e < NP * (n / 2); e += kBlock) {
            const int ql = e >> (LOGN - 1), j = e & (n / 2 - 1);
            const int k = j & (Ns - 1);
            const C a = src[ql * n + j];
            const C b0 = src[ql * n + j + n / 2];
            const C w = tw[k * (n / (2 * Ns))];
            C b;
            b.x = b0.x * w.x - b0.y * w.y;
            b.y = b0.x * w.y + b0.y * w.x;
            const int idx = ((j - k) << 1) + k;
            dst[ql * n + idx] = C{a.x + b.x, a.y + b.y};
            dst[ql * n + idx + Ns] = C{a.x - b.x, a.y - b.y};
        }
        __syncthreads();
        C *t = src; src = dst; dst = t;
    }
    for (int e = threadIdx.x; e < NP * n; e += kBlock) {
        const T f = bconv[e & (n - 1)];
        C v = src[e];
        v.x *= f; v.y *= f;
        src[e] = v;
    }
    __syncthreads();
    // inverse transform (conjugate twiddles, no 1/n: folded into bconv)
    for (int Ns = 1; Ns < n; Ns <<= 1) {
        for (int e = threadIdx.x; e < NP * (n / 2); e += kBlock) {
            const int ql = e >> (LOGN - 1), j = e & (n / 2 - 1);
            const int k = j & (Ns - 1);
            const C a = src[ql * n + j];
            const C b0 = src[ql * n + j + n / 2];
            const C w = tw[k * (n / (2 * Ns))];
            C b;
            b.x = b0.x * w.x + b0.y * w.y;
            b.y = b0.y * w.x - b0.x * w.y;
            const int idx = ((j - k) << 1) + k;
            dst[ql * n + idx] = C{a.x + b.x, a.y + b.y};
            dst[ql * n + idx + Ns] = C{a.x - b.x, a.y - b.y};
        }
        __syncthreads();
        C *t = src; src = dst; dst = t;
    }
    for (int e = threadIdx.x; e < NP * n; e += kBlock) {
        int ql, u;
        if (contiguous) { ql = e / n; u = e % n; } else { u = e / NP; ql = e % NP; }
        const int r0 = 2 * (q0 + ql), r1 = r0 + 1;
        const C v = src[ql * n + u];
        if (r0 < nlines) grid[base_of(r0) + (size_t)u * s] = v.x;
        if (r1 < nlines) grid[base_of(r1) + (size_t)u * s] = v.y;
    }
}

// ------------------------------------------------------------------ fill
__global__ __launch_bounds__(kBlock) void zero_kernel(uint4 *__restrict__ p, size_t n16) {
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n16;
         i += (size_t)gridDim.x * kBlock)
        p[i] = uint4{0u, 0u, 0u, 0u};
}

void launch_zero(void *p, size_t bytes, hipStream_t s) {
    // every buffer handed here is a multiple of 16 bytes (allocations are
    // rounded up by the plan)
    const size_t n16 = bytes / 16;
    if (n16 == 0) return;
    const int blocks = (int)std::min<size_t>((n16 + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(kBlock), 0, s, (uint4 *)p, n16);
    ANOVA_HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------------ dispatch
static size_t region_bytes(const WindowPlan &w, size_t elem) {
    const size_t L = (size_t)w.tile + 2 * w.m - 1;
    size_t v = L;
    if (w.dA >= 2) v *= L;
    if (w.dA >= 3) v *= L;
    return v * elem;
}

template <typename T, int DA, int W>
static void spread_t(const WindowPlan &w, const double *alpha, void *priv, hipStream_t s) {
    if (w.n_sub == 0) return;
    const size_t shm = region_bytes(w, sizeof(unsigned long long));
    hipLaunchKernelGGL((spread_kernel<T, DA, W>), dim3((unsigned)w.n_sub), dim3(kBlock), shm, s,
                       w.nodes.as<typename NodeOf<T>::type>(), w.perm.as<int32_t>(),
                       w.subs.as<SubProblem>(), alpha, (T *)priv, w.poly.as<T>(), w.poly_deg,
                       w.tile, w.tiles_per_dim);
    ANOVA_HIP_CHECK(hipGetLastError());
}

template <typename T, int DA>
static void fold_t(const WindowPlan &w, const void *priv, void *treg, void *grid, hipStream_t s) {
    const int vol = (int)w.region_elems();
    const void *src = priv;
    if (w.n_sub != w.n_nonempty) {
        hipLaunchKernelGGL((tile_sum_kernel<T>), dim3((vol + kBlock - 1) / kBlock, (unsigned)w.n_nonempty),
                           dim3(kBlock), 0, s, (const T *)priv, w.src_sub.as<int32_t>(), (T *)treg,
                           vol);
        ANOVA_HIP_CHECK(hipGetLastError());
        src = treg;
    }
    hipLaunchKernelGGL((fold_kernel<T, DA>), dim3((unsigned)w.n_tiles), dim3(kBlock), 0, s,
                       (const T *)src, w.fold_pairs.as<int2>(), w.fold_start.as<int32_t>(),
                       (T *)grid, w.n, w.tile, w.tiles_per_dim, w.tile + 2 * w.m - 1);
    ANOVA_HIP_CHECK(hipGetLastError());
}

template <typename T, int DA, int W>
static void gather_t(const WindowPlan &w, const void *grid, const double *alpha, double *out,
                     double beta, bool first, hipStream_t s) {
    if (w.n_sub == 0) return;
    const size_t shm = region_bytes(w, sizeof(T));
    if (first)
        hipLaunchKernelGGL((gather_kernel<T, DA, W, true>), dim3((unsigned)w.n_sub), dim3(kBlock),
                           shm, s, w.nodes.as<typename NodeOf<T>::type>(), w.perm.as<int32_t>(),
                           w.subs.as<SubProblem>(), (const T *)grid, alpha, out, w.eta, beta,
                           w.poly.as<T>(), w.poly_deg, w.n, w.tile, w.tiles_per_dim);
    else
        hipLaunchKernelGGL((gather_kernel<T, DA, W, false>), dim3((unsigned)w.n_sub), dim3(kBlock),
                           shm, s, w.nodes.as<typename NodeOf<T>::type>(), w.perm.as<int32_t>(),
                           w.subs.as<SubProblem>(), (const T *)grid, alpha, out, w.eta, beta,
                           w.poly.as<T>(), w.poly_deg, w.n, w.tile, w.tiles_per_dim);
    ANOVA_HIP_CHECK(hipGetLastError());
}

#define ANOVA_DISPATCH_W(DA, FN, ...)                                     \
    switch (w.m) {                                                        \
        case 2: FN<T, DA, 4>(__VA_ARGS__); break;                         \
        case 3: FN<T, DA, 6>(__VA_ARGS__); break;                         \
        case 4: FN<T, DA, 8>(__VA_ARGS__); break;                         \
        case 5: FN<T, DA, 10>(__VA_ARGS__); break;                        \
        case 6: FN<T, DA, 12>(__VA_ARGS__); break;                        \
        case 7: FN<T, DA, 14>(__VA_ARGS__); break;                        \
        case 8: FN<T, DA, 16>(__VA_ARGS__); break;                        \
        default: throw Error{ANOVA_E_INVALID, "window half-width m out of range"}; \
    }

template <typename T>
static void spread_typed(const WindowPlan &w, const double *alpha, void *priv, hipStream_t s) {
    switch (w.dA) {
        case 1: ANOVA_DISPATCH_W(1, spread_t, w, alpha, priv, s); break;
        case 2: ANOVA_DISPATCH_W(2, spread_t, w, alpha, priv, s); break;
        case 3: ANOVA_DISPATCH_W(3, spread_t, w, alpha, priv, s); break;
        default: throw Error{ANOVA_E_INVALID, "d_A out of range"};
    }
}

template <typename T>
static void fold_typed(const WindowPlan &w, const void *priv, void *treg, void *grid,
                       hipStream_t s) {
    switch (w.dA) {
        case 1: fold_t<T, 1>(w, priv, treg, grid, s); break;
        case 2: fold_t<T, 2>(w, priv, treg, grid, s); break;
        case 3: fold_t<T, 3>(w, priv, treg, grid, s); break;
        default: throw Error{ANOVA_E_INVALID, "d_A out of range"};
    }
}

template <typename T>
static void gather_typed(const WindowPlan &w, const void *grid, const double *alpha, double *out,
                         double beta, bool first, hipStream_t s) {
    switch (w.dA) {
        case 1: ANOVA_DISPATCH_W(1, gather_t, w, grid, alpha, out, beta, first, s); break;
        case 2: ANOVA_DISPATCH_W(2, gather_t, w, grid, alpha, out, beta, first, s); break;
        case 3: ANOVA_DISPATCH_W(3, gather_t, w, grid, alpha, out, beta, first, s); break;
        default: throw Error{ANOVA_E_INVALID, "d_A out of range"};
    }
}

void launch_spread_regions(const WindowPlan &w, int precision, const double *alpha, void *priv,
                           hipStream_t s) {
    if (precision == ANOVA_FP64)
        spread_typed<double>(w, alpha, priv, s);
    else
        spread_typed<float>(w, alpha, priv, s);
}

void launch_fold(const WindowPlan &w, int precision, const void *priv, void *treg, void *grid,
                 hipStream_t s) {
    if (precision == ANOVA_FP64)
        fold_typed<double>(w, priv, treg, grid, s);
    else
        fold_typed<float>(w, priv, treg, grid, s);
}

void launch_spread(const WindowPlan &w, int precision, const double *alpha, void *grid, void *priv,
                   void *treg, hipStream_t s) {
    launch_spread_regions(w, precision, alpha, priv, s);
    launch_fold(w, precision, priv, treg, grid, s);
}

void launch_gather(const WindowPlan &w, int precision, const void *grid, const double *alpha,
                   double *out, double beta, bool first, hipStream_t s) {
    if (precision == ANOVA_FP64)
        gather_typed<double>(w, grid, alpha, out, beta, first, s);
    else
        gather_typed<float>(w, grid, alpha, out, beta, first, s);
}

template <typename T, int LOGN>
static void convolve_axis(const WindowPlan &w, T *grid, int axis, hipStream_t s) {
    constexpr int n = 1 << LOGN;
    int nlines = 1;
    for (int t = 1; t < w.dA; ++t) nlines *= n;
    int stride = 1;
    for (int t = 0; t < axis; ++t) stride *= n;
    const int nq = (nlines + 1) / 2;
    // lines per workgroup: enough butterflies per stage to occupy the block,
    // but at least ~256 workgroups when the grid has that many lines
    const int per_block = std::max(1, 512 / n);
    const int NP = std::max(1, std::min(per_block, (nq + 255) / 256));
    const int blocks = (nq + NP - 1) / NP;
    const size_t shm = 2 * (size_t)NP * n * sizeof(typename Cplx<T>::type);
    hipLaunchKernelGGL((convolve_kernel<T, LOGN>), dim3(blocks), dim3(kBlock), shm, s, grid,
                       w.bconv.as<T>(), w.twiddle.as<typename Cplx<T>::type>(), nlines, stride,
                       NP);
    ANOVA_HIP_CHECK(hipGetLastError());
}

template <typename T>
static void convolve_typed(const WindowPlan &w, T *grid, hipStream_t s) {
    for (int axis = 0; axis < w.dA; ++axis) {
        switch (w.n) {
            case 8: convolve_axis<T, 3>(w, grid, axis, s); break;
            case 16: convolve_axis<T, 4>(w, grid, axis, s); break;
            case 32: convolve_axis<T, 5>(w, grid, axis, s); break;
            case 64: convolve_axis<T, 6>(w, grid, axis, s); break;
            case 128: convolve_axis<T, 7>(w, grid, axis, s); break;
            case 256: convolve_axis<T, 8>(w, grid, axis, s); break;
            default: throw Error{ANOVA_E_INVALID, "grid length n must be a power of two in [8, 256]"};
        }
    }
}

void launch_convolve(const WindowPlan &w, int precision, void *grid, hipStream_t s) {
    if (precision == ANOVA_FP64)
        convolve_typed<double>(w, (double *)grid, s);
    else
        convolve_typed<float>(w, (float *)grid, s);
}

}  // namespace anova
