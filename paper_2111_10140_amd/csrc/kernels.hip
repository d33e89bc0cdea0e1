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
// The degree is fixed per precision (kPolyDeg), so the loops unroll and the
// coefficients, uniform across the wave, stay in scalar registers.
template <typename T, int W>
__device__ __forceinline__ void window_weights(const T *__restrict__ poly, int /*deg*/, T f,
                                               T (&w)[W]) {
    constexpr int D = PolyDeg<T>::value;
    const T z = T(2) * f - T(1);
#pragma unroll
    for (int a = 0; a < W; ++a) w[a] = poly[a * (D + 1) + D];
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
#pragma unroll
        for (int a = 0; a < W; ++a) w[a] = w[a] * z + poly[a * (D + 1) + k];
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
    const typename NodeOf<T>::type *__restrict__ nodes, const T *__restrict__ as,
    const SubProblem *__restrict__ subs, T *__restrict__ priv, const T *__restrict__ poly,
    int deg, int tile, int tpd) {
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
        float va = (float)fabs(as[j]);
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
        const T a = as[j] * sc;
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

// ------------------------------------------------------------------ dense regime
// With many points per grid cell (float32, small support), points are sorted
// by cell inside each tile and thread (cell, s) handles points s, s+S, ... of
// its cell.  Spreading accumulates the cell's W^d_A support values in
// registers and adds them to the tile region once per thread; gathering reads
// the cell's support values from LDS once and interpolates every point of the
// thread.  One workgroup per non-empty tile (TILE^d_A cells, S threads each).
template <int DA, int TILE>
struct DenseShape {
    static constexpr int cells = DA == 3 ? TILE * TILE * TILE : (DA == 2 ? TILE * TILE : TILE);
};

template <int DA, int W, int TILE, int S>
__global__ __launch_bounds__(kBlock) void spread_dense_kernel(
    const NodeF32 *__restrict__ nodes, const float *__restrict__ as,
    const int32_t *__restrict__ tiles, const int32_t *__restrict__ cell_start,
    float *__restrict__ priv, const float *__restrict__ poly, int deg, int K) {
    constexpr int L = TILE + W - 1;
    constexpr int L2 = DA >= 2 ? L * L : L;
    constexpr int VOL = DA == 3 ? L2 * L : L2;
    constexpr int CELLS = DenseShape<DA, TILE>::cells;
    static_assert(CELLS * S == kBlock, "one thread per (cell, split)");
    constexpr int WY = DA >= 2 ? W : 1, WZ = DA == 3 ? W : 1;
    __shared__ unsigned long long acc_lds[VOL];
    __shared__ float red[kBlock / 64];
    const int tk = blockIdx.x / K, chunk = blockIdx.x % K;
    const int key0 = tiles[tk] * CELLS;
    for (int e = threadIdx.x; e < VOL; e += kBlock) acc_lds[e] = 0ull;
    const int cell = threadIdx.x / S;
    const int q = chunk * S + (int)(threadIdx.x % S), QS = K * S;
    const int lx = cell % TILE;
    const int ly = DA >= 2 ? (cell / TILE) % TILE : 0;
    const int lz = DA == 3 ? cell / (TILE * TILE) : 0;
    float acc[WZ][WY][W];
#pragma unroll
    for (int c = 0; c < WZ; ++c)
#pragma unroll
        for (int b = 0; b < WY; ++b)
#pragma unroll
            for (int i = 0; i < W; ++i) acc[c][b][i] = 0.0f;
    // the fixed-point scale is needed only for the final flush, so the
    // largest |coefficient| of the workgroup is tracked along the way
    float amax = 0.0f;
    const int c1 = cell_start[key0 + cell + 1];
    int j = cell_start[key0 + cell] + q;
    // software pipeline: the next point's record and coefficient load while
    // the current one is accumulated
    NodeF32 rec_n{};
    float a_n = 0.0f;
    if (j < c1) { rec_n = nodes[j]; a_n = as[j]; }
    for (; j < c1; j += QS) {
        const NodeF32 rec = rec_n;
        const float a = a_n;
        if (j + QS < c1) { rec_n = nodes[j + QS]; a_n = as[j + QS]; }
        float va = fabsf(a);
        if (!(va <= 3.0e38f)) va = INFINITY;
        amax = fmaxf(amax, va);
        float wx[W], wy[W], wz[W];
        window_weights<float, W>(poly, deg, rec.f[0], wx);
        if constexpr (DA >= 2) window_weights<float, W>(poly, deg, rec.f[1], wy);
        if constexpr (DA == 3) window_weights<float, W>(poly, deg, rec.f[2], wz);
#pragma unroll
        for (int c = 0; c < WZ; ++c) {
            const float wc = DA == 3 ? a * wz[c] : a;
#pragma unroll
            for (int b = 0; b < WY; ++b) {
                const float wbc = DA >= 2 ? wc * wy[b] : wc;
#pragma unroll
                for (int i = 0; i < W; ++i) acc[c][b][i] = fmaf(wbc, wx[i], acc[c][b][i]);
            }
        }
    }
    amax = block_max(amax, red);  // also orders the zero fill before the adds
    float *out = priv + (size_t)blockIdx.x * VOL;
    if (!(amax > 0.0f) || !isfinite(amax)) {
        const float fill = amax > 0.0f ? NAN : 0.0f;
        for (int e = threadIdx.x; e < VOL; e += kBlock) out[e] = fill;
        return;
    }
    int ex2;
    (void)frexpf(amax * 1.0000002f, &ex2);
    const int Sx = 30 - ex2;
    const double sc = ldexp(1.0, Sx);
#pragma unroll
    for (int c = 0; c < WZ; ++c)
#pragma unroll
        for (int b = 0; b < WY; ++b)
#pragma unroll
            for (int i = 0; i < W; ++i) {
                const float v = acc[c][b][i];
                if (v != 0.0f)
                    atomicAdd(&acc_lds[((lz + c) * L + ly + b) * L + lx + i],
                              (unsigned long long)round_to_ll((double)v * sc));
            }
    __syncthreads();
    const double inv = ldexp(1.0, -Sx);
    for (int e = threadIdx.x; e < VOL; e += kBlock)
        out[e] = (float)((double)(long long)acc_lds[e] * inv);
}

template <int DA, int W, int TILE, int S>
__global__ __launch_bounds__(kBlock) void gather_dense_kernel(
    const NodeF32 *__restrict__ nodes, const int32_t *__restrict__ tiles,
    const int32_t *__restrict__ cell_start, const float *__restrict__ grid,
    float *__restrict__ tmp, const float *__restrict__ poly, int deg, int n, int tpd, int K) {
    constexpr int m = W / 2;
    constexpr int L = TILE + W - 1;
    constexpr int L2 = DA >= 2 ? L * L : L;
    constexpr int VOL = DA == 3 ? L2 * L : L2;
    constexpr int CELLS = DenseShape<DA, TILE>::cells;
    static_assert(CELLS * S == kBlock, "one thread per (cell, split)");
    constexpr int WY = DA >= 2 ? W : 1, WZ = DA == 3 ? W : 1;
    __shared__ float g_lds[VOL];
    const int chunk = blockIdx.x % K;
    const int tile_id = tiles[blockIdx.x / K];
    const int key0 = tile_id * CELLS;
    const int ox = (tile_id % tpd) * TILE;
    const int oy = ((tile_id / tpd) % tpd) * TILE;
    const int oz = (tile_id / (tpd * tpd)) * TILE;
    for (int e = threadIdx.x; e < VOL; e += kBlock) {
        const int ex = e % L;
        size_t g = (size_t)wrap_index(ox - m + 1 + ex, n);
        if constexpr (DA >= 2) g += (size_t)n * (size_t)wrap_index(oy - m + 1 + (e / L) % L, n);
        if constexpr (DA == 3) g += (size_t)n * (size_t)n * (size_t)wrap_index(oz - m + 1 + e / L2, n);
        g_lds[e] = grid[g];
    }
    __syncthreads();
    const int cell = threadIdx.x / S;
    const int q = chunk * S + (int)(threadIdx.x % S), QS = K * S;
    const int lx = cell % TILE;
    const int ly = DA >= 2 ? (cell / TILE) % TILE : 0;
    const int lz = DA == 3 ? cell / (TILE * TILE) : 0;
    const int c0 = cell_start[key0 + cell] + q, c1 = cell_start[key0 + cell + 1];
    if (c0 >= c1) return;
    float g[WZ][WY][W];
#pragma unroll
    for (int c = 0; c < WZ; ++c)
#pragma unroll
        for (int b = 0; b < WY; ++b)
#pragma unroll
            for (int i = 0; i < W; ++i) g[c][b][i] = g_lds[((lz + c) * L + ly + b) * L + lx + i];
    for (int j = c0; j < c1; j += QS) {
        const NodeF32 rec = nodes[j];
        float wx[W], wy[W], wz[W];
        window_weights<float, W>(poly, deg, rec.f[0], wx);
        if constexpr (DA >= 2) window_weights<float, W>(poly, deg, rec.f[1], wy);
        if constexpr (DA == 3) window_weights<float, W>(poly, deg, rec.f[2], wz);
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < WZ; ++c) {
            float sc = 0.0f;
#pragma unroll
            for (int b = 0; b < WY; ++b) {
                float s = 0.0f;
#pragma unroll
                for (int i = 0; i < W; ++i) s = fmaf(g[c][b][i], wx[i], s);
                sc = DA >= 2 ? fmaf(s, wy[b], sc) : s;
            }
            acc = DA == 3 ? fmaf(sc, wz[c], acc) : sc;
        }
        tmp[j] = acc;
    }
}

// ------------------------------------------------------------------ permute
// Coefficients in the window's sorted point order: as[j] = alpha[perm[j]].
template <typename T>
__global__ __launch_bounds__(kBlock) void permute_kernel(const double *__restrict__ alpha,
                                                         const int32_t *__restrict__ perm,
                                                         T *__restrict__ as, int N) {
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < N; j += gridDim.x * kBlock)
        as[j] = static_cast<T>(alpha[perm[j]]);
}

// ------------------------------------------------------------------ combine
// out_i = beta alpha_i + sum_l eta_l tmp_l[iperm_l[i]] in float64, windows
// in order (accumulate: out_i += ... instead).  tmp_l holds window l's
// interpolated values in its sorted point order, iperm_l maps the caller's
// point index to that order.
template <typename T>
__global__ __launch_bounds__(kBlock) void combine_kernel(const CombineWin *__restrict__ wins,
                                                         int P, const double *__restrict__ alpha,
                                                         double *__restrict__ out, double beta,
                                                         int N, int accumulate) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
        double s = accumulate ? out[i] : beta * alpha[i];
        for (int l = 0; l < P; ++l) {
            const CombineWin cw = wins[l];
            s += cw.eta * (double)static_cast<const T *>(cw.tmp)[cw.iperm[i]];
        }
        out[i] = s;
    }
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
template <typename T, int DA, int W>
__global__ __launch_bounds__(kBlock) void gather_kernel(
    const typename NodeOf<T>::type *__restrict__ nodes, const SubProblem *__restrict__ subs,
    const T *__restrict__ grid, T *__restrict__ tmp, const T *__restrict__ poly, int deg, int n,
    int tile, int tpd) {
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
        tmp[j] = acc;
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
static void spread_t(const WindowPlan &w, const void *as, void *priv, hipStream_t s) {
    if (w.n_sub == 0) return;
    const size_t shm = region_bytes(w, sizeof(unsigned long long));
    hipLaunchKernelGGL((spread_kernel<T, DA, W>), dim3((unsigned)w.n_sub), dim3(kBlock), shm, s,
                       w.nodes.as<typename NodeOf<T>::type>(), (const T *)as,
                       w.subs.as<SubProblem>(), (T *)priv, w.poly.as<T>(), w.poly_deg, w.tile,
                       w.tiles_per_dim);
    ANOVA_HIP_CHECK(hipGetLastError());
}

template <typename T, int DA>
static void fold_t(const WindowPlan &w, const void *priv, void *treg, void *grid, hipStream_t s) {
    const int vol = (int)w.region_elems();
    const void *src = priv;
    if (w.n_regions != w.n_nonempty) {
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
static void gather_t(const WindowPlan &w, const void *grid, void *tmp, hipStream_t s) {
    if (w.n_sub == 0) return;
    const size_t shm = region_bytes(w, sizeof(T));
    hipLaunchKernelGGL((gather_kernel<T, DA, W>), dim3((unsigned)w.n_sub), dim3(kBlock), shm, s,
                       w.nodes.as<typename NodeOf<T>::type>(), w.subs.as<SubProblem>(),
                       (const T *)grid, (T *)tmp, w.poly.as<T>(), w.poly_deg, w.n, w.tile,
                       w.tiles_per_dim);
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

// dense-regime launches: tile edge 4 / 16 / 64 for d_A = 3 / 2 / 1 and
// 256 / cells threads per cell; supports up to W = 6 / 8 / 16
template <int DA>
struct DenseTile {
    static constexpr int value = DA == 3 ? 4 : (DA == 2 ? 16 : 64);
};
template <int DA, int W>
static constexpr bool dense_supported() {
    return DA == 3 ? W <= 6 : (DA == 2 ? W <= 8 : W <= 16);
}

template <int DA, int W>
static void spread_dense_t(const WindowPlan &w, const void *as, void *priv, hipStream_t s) {
    if constexpr (dense_supported<DA, W>()) {
        constexpr int TILE = DenseTile<DA>::value;
        constexpr int S = kBlock / DenseShape<DA, TILE>::cells;
        if (w.n_nonempty == 0) return;
        hipLaunchKernelGGL((spread_dense_kernel<DA, W, TILE, S>),
                           dim3((unsigned)(w.n_nonempty * w.chunks)), dim3(kBlock), 0, s,
                           w.nodes.as<NodeF32>(), (const float *)as, w.tiles_ne.as<int32_t>(),
                           w.cell_start.as<int32_t>(), (float *)priv, w.poly.as<float>(),
                           w.poly_deg, w.chunks);
        ANOVA_HIP_CHECK(hipGetLastError());
    } else {
        throw Error{ANOVA_E_INVALID, "dense spreading does not support this window width"};
    }
}

template <int DA, int W>
static void gather_dense_t(const WindowPlan &w, const void *grid, void *tmp, hipStream_t s) {
    if constexpr (dense_supported<DA, W>()) {
        constexpr int TILE = DenseTile<DA>::value;
        constexpr int S = kBlock / DenseShape<DA, TILE>::cells;
        if (w.n_nonempty == 0) return;
        hipLaunchKernelGGL((gather_dense_kernel<DA, W, TILE, S>),
                           dim3((unsigned)(w.n_nonempty * w.chunks)), dim3(kBlock), 0, s,
                           w.nodes.as<NodeF32>(), w.tiles_ne.as<int32_t>(),
                           w.cell_start.as<int32_t>(), (const float *)grid, (float *)tmp,
                           w.poly.as<float>(), w.poly_deg, w.n, w.tiles_per_dim, w.chunks);
        ANOVA_HIP_CHECK(hipGetLastError());
    } else {
        throw Error{ANOVA_E_INVALID, "dense gathering does not support this window width"};
    }
}

#define ANOVA_DISPATCH_DENSE(DA, FN, ...)                                 \
    switch (w.m) {                                                        \
        case 2: FN<DA, 4>(__VA_ARGS__); break;                            \
        case 3: FN<DA, 6>(__VA_ARGS__); break;                            \
        case 4: FN<DA, 8>(__VA_ARGS__); break;                            \
        case 5: FN<DA, 10>(__VA_ARGS__); break;                           \
        case 6: FN<DA, 12>(__VA_ARGS__); break;                           \
        case 7: FN<DA, 14>(__VA_ARGS__); break;                           \
        case 8: FN<DA, 16>(__VA_ARGS__); break;                           \
        default: throw Error{ANOVA_E_INVALID, "window half-width m out of range"}; \
    }

static void spread_dense(const WindowPlan &w, const void *as, void *priv, hipStream_t s) {
    switch (w.dA) {
        case 1: ANOVA_DISPATCH_DENSE(1, spread_dense_t, w, as, priv, s); break;
        case 2: ANOVA_DISPATCH_DENSE(2, spread_dense_t, w, as, priv, s); break;
        case 3: ANOVA_DISPATCH_DENSE(3, spread_dense_t, w, as, priv, s); break;
        default: throw Error{ANOVA_E_INVALID, "d_A out of range"};
    }
}

static void gather_dense(const WindowPlan &w, const void *grid, void *tmp, hipStream_t s) {
    switch (w.dA) {
        case 1: ANOVA_DISPATCH_DENSE(1, gather_dense_t, w, grid, tmp, s); break;
        case 2: ANOVA_DISPATCH_DENSE(2, gather_dense_t, w, grid, tmp, s); break;
        case 3: ANOVA_DISPATCH_DENSE(3, gather_dense_t, w, grid, tmp, s); break;
        default: throw Error{ANOVA_E_INVALID, "d_A out of range"};
    }
}

template <typename T>
static void spread_typed(const WindowPlan &w, const void *as, void *priv, hipStream_t s) {
    switch (w.dA) {
        case 1: ANOVA_DISPATCH_W(1, spread_t, w, as, priv, s); break;
        case 2: ANOVA_DISPATCH_W(2, spread_t, w, as, priv, s); break;
        case 3: ANOVA_DISPATCH_W(3, spread_t, w, as, priv, s); break;
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
static void gather_typed(const WindowPlan &w, const void *grid, void *tmp, hipStream_t s) {
    switch (w.dA) {
        case 1: ANOVA_DISPATCH_W(1, gather_t, w, grid, tmp, s); break;
        case 2: ANOVA_DISPATCH_W(2, gather_t, w, grid, tmp, s); break;
        case 3: ANOVA_DISPATCH_W(3, gather_t, w, grid, tmp, s); break;
        default: throw Error{ANOVA_E_INVALID, "d_A out of range"};
    }
}

void launch_spread_regions(const WindowPlan &w, int precision, const double *alpha, void *as,
                           void *priv, hipStream_t s) {
    const int N = (int)w.n_points;
    const int blocks = std::max(1, std::min((N + kBlock - 1) / kBlock, 4096));
    if (precision == ANOVA_FP64)
        hipLaunchKernelGGL(permute_kernel<double>, dim3(blocks), dim3(kBlock), 0, s, alpha,
                           w.perm.as<int32_t>(), (double *)as, N);
    else
        hipLaunchKernelGGL(permute_kernel<float>, dim3(blocks), dim3(kBlock), 0, s, alpha,
                           w.perm.as<int32_t>(), (float *)as, N);
    ANOVA_HIP_CHECK(hipGetLastError());
    if (w.dense)
        spread_dense(w, as, priv, s);
    else if (precision == ANOVA_FP64)
        spread_typed<double>(w, as, priv, s);
    else
        spread_typed<float>(w, as, priv, s);
}

void launch_fold(const WindowPlan &w, int precision, const void *priv, void *treg, void *grid,
                 hipStream_t s) {
    if (precision == ANOVA_FP64)
        fold_typed<double>(w, priv, treg, grid, s);
    else
        fold_typed<float>(w, priv, treg, grid, s);
}

void launch_spread(const WindowPlan &w, int precision, const double *alpha, void *grid, void *as,
                   void *priv, void *treg, hipStream_t s) {
    launch_spread_regions(w, precision, alpha, as, priv, s);
    launch_fold(w, precision, priv, treg, grid, s);
}

void launch_gather(const WindowPlan &w, int precision, const void *grid, void *tmp,
                   hipStream_t s) {
    if (w.dense)
        gather_dense(w, grid, tmp, s);
    else if (precision == ANOVA_FP64)
        gather_typed<double>(w, grid, tmp, s);
    else
        gather_typed<float>(w, grid, tmp, s);
}

void launch_combine(const void *wins, int P, int precision, const double *alpha, double *out,
                    double beta, int64_t N, bool accumulate, hipStream_t s) {
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((N + kBlock - 1) / kBlock, 8192));
    if (precision == ANOVA_FP64)
        hipLaunchKernelGGL(combine_kernel<double>, dim3(blocks), dim3(kBlock), 0, s,
                           (const CombineWin *)wins, P, alpha, out, beta, (int)N,
                           accumulate ? 1 : 0);
    else
        hipLaunchKernelGGL(combine_kernel<float>, dim3(blocks), dim3(kBlock), 0, s,
                           (const CombineWin *)wins, P, alpha, out, beta, (int)N,
                           accumulate ? 1 : 0);
    ANOVA_HIP_CHECK(hipGetLastError());
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
