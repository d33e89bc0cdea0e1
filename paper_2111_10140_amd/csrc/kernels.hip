// Hot-path kernels of the windows' fast summation (gfx950, wave64):
//   spread   : first step of the adjoint NFFT (Sec. 4.1, eq. adjnfft) --
//              point coefficients are spread onto the oversampled grid with a
//              compactly supported window;
//   convolve : d_A-dimensional FFT, multiplication by the kernel's Fourier
//              coefficients over the window transform squared, inverse FFT
//              (Sec. 4.2, eq. fastsum); the multiplier is a product over
//              dimensions, so the three steps factor into one
//              forward-FFT / multiply / inverse-FFT pass per axis;
//   gather   : last step of the NFFT (Sec. 4.1, eq. nfft) -- the grid is
//              interpolated back at the points with the same window;
//   combine  : sum over windows with weights eta_l (Sec. 5, K = sum eta_l K_l)
//              plus the shift beta alpha, in float64.
//
// Every kernel serves a list of "instances" (one window of one problem for
// one right-hand side, described by a WinInst in device memory): a launch
// covers all instances of one kernel signature, and each workgroup finds its
// instance by a binary search over the per-instance block counts.
//
// Points are sorted by grid tile at plan time.  Spreading forms one tile
// region (tile + halo of 2m-1 points) per workgroup -- per cell from
// registers with fixed-order sums (per-cell kernels), or in LDS with integer
// atomics (per-point kernels) -- and stores it with plain stores; a fold
// kernel adds the regions into the grid in a fixed order.  No floating-point
// atomics are used, so a product is bitwise reproducible.  Gathering writes
// each point's value at its position in the caller's order.
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "anova_internal.h"

namespace anova {

template <typename T> struct NodeOf;
template <> struct NodeOf<float> { using type = NodeF32; };
template <> struct NodeOf<double> { using type = NodeF64; };
template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

constexpr int kBlock = 256;

// Index q of the group member owning block b: prefix[q] <= b < prefix[q+1].
__device__ __forceinline__ int find_member(const int32_t *__restrict__ prefix, int cnt, int b) {
    int lo = 0, hi = cnt;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

struct Located {
    const WinInst *w;
    int lb;  // block index inside the instance
};

// The search depends on blockIdx only; readfirstlane makes the index (and so
// every instance field loaded through it) wave-uniform, i.e. scalar.
__device__ __forceinline__ Located locate(const WinInst *__restrict__ insts,
                                          const int32_t *__restrict__ members,
                                          const int32_t *__restrict__ prefix, int cnt) {
    const int b = blockIdx.x;
    const int q = __builtin_amdgcn_readfirstlane(find_member(prefix, cnt, b));
    const int mi = __builtin_amdgcn_readfirstlane(members[q]);
    return Located{insts + mi, b - __builtin_amdgcn_readfirstlane(prefix[q])};
}

__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Weights phi0(f + m - 1 - a), a = 0..W-1, of a point with fractional cell
// offset f in [0,1): one polynomial per support offset, Horner in z = 2f-1.
// The degree is fixed per precision and width, so the loops unroll and the
// coefficients, uniform across the wave, stay in scalar registers.
template <typename T, int W>
__device__ __forceinline__ void window_weights(const T *__restrict__ poly, T f, T (&w)[W]) {
    constexpr int D = PolyDeg<T>::of(W);
    const T z = T(2) * f - T(1);
#pragma unroll
    for (int a = 0; a < W; ++a) w[a] = poly[a * (D + 1) + D];
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
#pragma unroll
        for (int a = 0; a < W; ++a) w[a] = w[a] * z + poly[a * (D + 1) + k];
    }
}

// The window polynomials held in registers for a whole kernel (the kernels
// store to global memory inside their loops, so reading the table through a
// pointer there would be reloaded after every store).  The window is even,
// so the polynomial of offset W-1-a at z equals that of offset a at -z:
// only the lower half is held, and split into its even and odd parts in z,
// p(z) = E(z^2) + z O(z^2), it gives both weights of the pair (a, W-1-a),
// E + zO and E - zO, for about half the multiply-adds of two evaluations.
template <typename T, int W, int DEG = PolyDeg<T>::of(W)>
struct WinPoly {
    static constexpr int D = DEG, H = W / 2;
    static_assert(W % 2 == 0, "supports of 2m points");
    T c[H][D + 1];
    __device__ __forceinline__ void load(const T *__restrict__ poly) {
#pragma unroll
        for (int a = 0; a < H; ++a)
#pragma unroll
            for (int k = 0; k <= D; ++k) c[a][k] = uniform(poly[a * (D + 1) + k]);
    }
    // weights of offsets a and W-1-a at z (z2 = z * z)
    __device__ __forceinline__ void pair(T z, T z2, int a, T &lo, T &hi) const {
        constexpr int KE = D - D % 2, KO = D - 1 + D % 2;  // highest even / odd power
        T e = c[a][KE], o = c[a][KO];
#pragma unroll
        for (int k = KE - 2; k >= 0; k -= 2) e = e * z2 + c[a][k];
#pragma unroll
        for (int k = KO - 2; k >= 1; k -= 2) o = o * z2 + c[a][k];
        lo = e + z * o;
        hi = e - z * o;
    }
    __device__ __forceinline__ void eval(T f, T (&w)[W]) const {
        const T z = T(2) * f - T(1), z2 = z * z;
#pragma unroll
        for (int a = 0; a < H; ++a) pair(z, z2, a, w[a], w[W - 1 - a]);
    }
    // weight of offset a < W/2 alone at z (offset W-1-a: at -z)
    __device__ __forceinline__ T at(T z, int a) const {
        T v = c[a][D];
#pragma unroll
        for (int k = D - 1; k >= 0; --k) v = v * z + c[a][k];
        return v;
    }
};

// The three fractional offsets of a float32 node record (its packed cell
// word is not needed by the per-cell kernels).
__device__ __forceinline__ float3 node_offsets(const NodeF32 *__restrict__ p) {
    return *reinterpret_cast<const float3 *>(p);
}

// Thread-strided fill of count LDS entries from global memory, U loads in
// flight per thread: load(e) reads entry e through a global view and is
// called for every e of a round (indices past the end clamped to the last,
// read again and dropped) before store(e, v) writes the round's entries.
template <int U, typename T, typename Load, typename Store>
__device__ __forceinline__ void fill_lds(int count, int nthreads, Load load, Store store) {
    for (int e0 = (int)threadIdx.x; e0 < count; e0 += U * nthreads) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = load(min(e0 + u * nthreads, count - 1));
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e0 + u * nthreads < count) store(e0 + u * nthreads, v[u]);
    }
}

// Offsets of float32 node record k through a global view of the records.
__device__ __forceinline__ float3 node_offsets(global_ptr<float> nf, int k) {
    const size_t b = 4 * (size_t)k;
    return make_float3(nf[b], nf[b + 1], nf[b + 2]);
}

// Periodic index on a grid of n points: n is a power of two (the plan
// requires it), so the two's-complement mask also wraps negative g.
__device__ __forceinline__ int wrap_index(int g, int n) { return g & (n - 1); }

// ------------------------------------------------------------------ fixed point
// LDS float atomics are slow on this chip while 64-bit integer LDS atomics
// run at full rate, and integer sums are exact: a contribution v is rounded
// to an integer at the workgroup's scale 2^S, chosen from the largest |alpha|
// of its points so that no contribution exceeds 2^30 (float32 path, rounding
// 2^-31 of max|alpha|) or 2^50 (float64 path, rounding 2^-51) in magnitude
// (window weights are at most 1); the int64 sum of
// at most 1024 such terms (a sub-problem's points, or the register sums of a
// tile's threads, each already scaled below 2^30) cannot overflow, and it
// does not depend on the order of the additions.
__device__ __forceinline__ long long round_to_ll(float x) {  // |x| < 2^31
    return (long long)__float2int_rn(x);
}
__device__ __forceinline__ long long round_to_ll(double x) {  // |x| < 2^51
    // x + 1.5 * 2^52 lies in (2^52, 2^53), where the spacing of doubles is 1:
    // the addition rounds x to the nearest integer (ties to even) and the
    // low mantissa bits then hold it, offset by those of 1.5 * 2^52
    const double t = x + 0x1.8p52;
    return __double_as_longlong(t) - __double_as_longlong(0x1.8p52);
}
template <typename T> struct FixedBits;
template <> struct FixedBits<float> { static constexpr int value = 30; };
template <> struct FixedBits<double> { static constexpr int value = 50; };

__device__ __forceinline__ float block_max(float v, float *sh) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    float r = sh[0];
    for (int i = 1; i < kBlock / 64; ++i) r = fmaxf(r, sh[i]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double *sh) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
    for (int i = 1; i < kBlock / 64; ++i) r = fmax(r, sh[i]);
    __syncthreads();
    return r;
}

// Sum over the workgroup (kBlock threads) in a fixed order; valid in
// thread 0.  sh: kBlock / 64 doubles of LDS.
__device__ __forceinline__ double block_sum_f64(double v, double *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) t += sh[i];
    __syncthreads();
    return t;
}

// |a| for the largest-coefficient search of the float32 kernels: values
// beyond the float range (and NaN) become infinity, which marks the region
// as non-finite.
__device__ __forceinline__ float abs_for_max(double a) {
    const float va = (float)fabs(a);
    return va <= 3.0e38f ? va : INFINITY;
}
// The float64 kernels search in float64, so every finite coefficient,
// however small or large, sets a finite scale.
__device__ __forceinline__ double abs_for_max64(double a) {
    return fabs(a) <= 1.79e308 ? fabs(a) : INFINITY;
}

// Region of a workgroup with non-finite or all-zero coefficients.
template <typename T, typename A>
__device__ __forceinline__ bool trivial_region(A amax, T *out, int vol) {
    if (amax > A(0) && isfinite(amax)) return false;
    const T fill = amax > A(0) ? T(NAN) : T(0);
    for (int e = threadIdx.x; e < vol; e += kBlock) out[e] = fill;
    return true;
}

// Exponent e with amax (1 + margin) < 2^e, for the fixed-point scale.
__device__ __forceinline__ int scale_exponent(float amax) {
    int e;
    (void)frexpf(amax * 1.0000002f, &e);
    return e;
}
__device__ __forceinline__ int scale_exponent(double amax) {
    int e;
    (void)frexp(amax * (1.0 + 0x1p-40), &e);
    return e;
}

// ------------------------------------------------------------------ spread, per point
// One workgroup per sub-problem (a run of at most 1024 points of one tile).
template <typename T, int DA, int W>
__global__ __launch_bounds__(kBlock) void spread_pt_kernel(const WinInst *__restrict__ insts,
                                                           const int32_t *__restrict__ members,
                                                           const int32_t *__restrict__ prefix,
                                                           int cnt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem_raw);
    // the largest |coefficient| is searched in float32 on the float32 path
    // (its coefficients are floats) and in float64 on the float64 path
    using AM = typename std::conditional<std::is_same<T, double>::value, double, float>::type;
    __shared__ AM red[kBlock / 64];
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    using Node = typename NodeOf<T>::type;
    const Node *__restrict__ nodes = static_cast<const Node *>(wi.nodes);
    const T *__restrict__ as = static_cast<const T *>(wi.tmp);  // sorted coefficients
    const T *__restrict__ poly = static_cast<const T *>(wi.poly);
    const int tile = wi.tile, tpd = wi.tpd;
    const int L = tile + W - 1;
    const int L2 = DA >= 2 ? L * L : L;
    const int vol = DA == 3 ? L2 * L : L2;
    for (int e = threadIdx.x; e < vol; e += kBlock) acc[e] = 0ull;
    const SubProblem sp = wi.subs[loc.lb];
    const int end = sp.start + sp.count;
    AM amax = AM(0);
    for (int j = sp.start + threadIdx.x; j < end; j += kBlock) {
        if constexpr (std::is_same<T, double>::value) amax = fmax(amax, abs_for_max64(as[j]));
        else amax = fmaxf(amax, abs_for_max((double)as[j]));
    }
    amax = block_max(amax, red);  // also orders the zero fill before the adds
    T *out = static_cast<T *>(wi.priv) + (size_t)loc.lb * vol;
    if (trivial_region(amax, out, vol)) return;
    const int S = FixedBits<T>::value - scale_exponent(amax);
    const int ox = (sp.tile % tpd) * tile;
    const int oy = ((sp.tile / tpd) % tpd) * tile;
    const int oz = (sp.tile / (tpd * tpd)) * tile;
    for (int j = sp.start + threadIdx.x; j < end; j += kBlock) {
        const Node rec = nodes[j];
        const T a = ldexp(as[j], S);  // |a| < 2^FixedBits
        const int lx = int(rec.cell & 1023u) - ox;
        T wx[W];
        window_weights<T, W>(poly, rec.f[0], wx);
        if constexpr (DA == 1) {
#pragma unroll
            for (int i = 0; i < W; ++i)
                atomicAdd(&acc[lx + i], (unsigned long long)round_to_ll(a * wx[i]));
        } else {
            const int ly = int((rec.cell >> 10) & 1023u) - oy;
            T wy[W];
            window_weights<T, W>(poly, rec.f[1], wy);
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
                window_weights<T, W>(poly, rec.f[2], wz);
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
    // ldexp rather than a product with 2^-S: S can exceed 1022 for float64
    // coefficients near the bottom of the range, where 2^-S is no longer a
    // normal double
    for (int e = threadIdx.x; e < vol; e += kBlock)
        out[e] = static_cast<T>(ldexp((double)(long long)acc[e], -S));
}

// ------------------------------------------------------------------ per-cell kernels
// With many points per grid cell (float32, small support), points are sorted
// by cell inside each tile; chunk k of K takes a contiguous range of each
// cell's points and thread (cell, s) of the chunk handles points s, s + S,
// ... of that range.  Spreading accumulates the cell's W^d_A support values
// in registers and adds them to the tile region once per thread; gathering
// reads the cell's support values from LDS once and interpolates every
// point of the thread.  Workgroups: non-empty tiles x K.
// Points of chunk k of K of a cell [cs, ce): a contiguous range, so that
// the lines of the sorted records and values a workgroup touches are
// consumed by that workgroup over consecutive iterations (neighbouring
// chunks usually run on other XCDs, whose L2 caches are separate).
__device__ __forceinline__ void chunk_range(int cs, int ce, int k, int K, int &b, int &e) {
    const long long cnt = ce - cs;
    b = cs + (int)(cnt * k / K);
    e = cs + (int)(cnt * (k + 1) / K);
}

// Workgroup lb of a per-cell launch: its non-empty tile k (chunk_start =
// src_sub, ascending), its chunk inside the tile and the tile's chunk count.
// Plans give every tile of a window the same count (chunks > 0), so the
// tile is lb / chunks with no load at all; a search over the starts
// otherwise.
__device__ __forceinline__ void locate_chunk(const int32_t *__restrict__ cstart, int n_ne, int chunks,
                                             int lb, int &k, int &chunk, int &K) {
    if (chunks > 0) {
        k = __builtin_amdgcn_readfirstlane(lb / chunks);
        K = chunks;
        chunk = lb - k * chunks;
        return;
    }
    int lo = 0, hi = n_ne;  // cstart[lo] <= lb < cstart[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cstart[mid] <= lb) lo = mid; else hi = mid;
    }
    k = __builtin_amdgcn_readfirstlane(lo);
    const int c0 = __builtin_amdgcn_readfirstlane(cstart[k]);
    K = __builtin_amdgcn_readfirstlane(cstart[k + 1]) - c0;
    chunk = lb - c0;
}

template <int DA, int TILE>
struct CellShape {
    static constexpr int cells = DA == 3 ? TILE * TILE * TILE : (DA == 2 ? TILE * TILE : TILE);
};

// Steps of a sum over the four lanes of a quad (lanes 4c .. 4c+3) with DPP
// quad permutations: after both steps every lane of the quad holds the same
// bits (each step adds two values, and float addition is commutative).  All
// four lanes must be active.
__device__ __forceinline__ float quad_step1(float v) {  // + lane ^ 1
    return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float quad_step2(float v) {  // + lane ^ 2
    return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
}

// Spreading per cell.  After the point loop, the S splits of a cell are
// summed across their lanes, the cells' W^d_A register tiles are staged in
// LDS, and each thread forms the region values it owns by adding the staged
// contributions of every cell whose support covers them, in a fixed order.
// No atomics: the region is the same bits for any scheduling.
template <int DA, int W, int TILE, int S>
__global__ __launch_bounds__(kBlock) void spread_cell_kernel(const WinInst *__restrict__ insts,
                                                             const int32_t *__restrict__ members,
                                                             const int32_t *__restrict__ prefix,
                                                             int cnt) {
    constexpr int L = TILE + W - 1;
    constexpr int L2 = DA >= 2 ? L * L : L;
    constexpr int VOL = DA == 3 ? L2 * L : L2;
    constexpr int CELLS = CellShape<DA, TILE>::cells;
    static_assert(CELLS * S == kBlock, "one thread per (cell, split)");
    static_assert(S == 1 || S == 4, "splits of a cell are summed within a quad");
    constexpr int WY = DA >= 2 ? W : 1, WZ = DA == 3 ? W : 1;
    constexpr int VW = WZ * WY * W;  // support values of one cell
    __shared__ __align__(16) float stage[CELLS * VW];
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    const NodeF32 *__restrict__ nodes = static_cast<const NodeF32 *>(wi.nodes);
    WinPoly<float, W> wp;
    wp.load(static_cast<const float *>(wi.poly));
    int tk, chunk, K;
    locate_chunk(wi.src_sub, wi.n_nonempty, wi.chunks, loc.lb, tk, chunk, K);
    const int key0 = wi.tiles_ne[tk] * CELLS;
    const int cell = threadIdx.x / S, split = (int)(threadIdx.x % S);
    int pb, pe;
    chunk_range(wi.cell_start[key0 + cell], wi.cell_start[key0 + cell + 1], chunk, K, pb, pe);
    float acc[WZ][WY][W];
#pragma unroll
    for (int c = 0; c < WZ; ++c)
#pragma unroll
        for (int b = 0; b < WY; ++b)
#pragma unroll
            for (int i = 0; i < W; ++i) acc[c][b][i] = 0.0f;
    const int c1 = pe;
    int j = pb + split;
    // software pipeline: the next point's offsets and coefficient (read in
    // the caller's order through the permutation, whose index loads one
    // point earlier still) load while the current one is accumulated, so
    // the scattered coefficient reads overlap the arithmetic
    const int32_t *__restrict__ perm = wi.perm;
    const double *__restrict__ alpha = wi.alpha;
    float3 r_n{};
    float a_n = 0.0f;
    int p_n = 0;
    if (j < c1) {
        r_n = node_offsets(nodes + j);
        a_n = (float)alpha[perm[j]];
    }
    if (j + S < c1) p_n = perm[j + S];
    for (; j < c1; j += S) {
        const float3 r = r_n;
        const float a = a_n;
        if (j + S < c1) {
            r_n = node_offsets(nodes + j + S);
            a_n = (float)alpha[p_n];
        }
        if (j + 2 * S < c1) p_n = perm[j + 2 * S];
        // z weights plane by plane: fewer live registers
        float wx[W], wy[W];
        wp.eval(r.x, wx);
        if constexpr (DA >= 2) wp.eval(r.y, wy);
        const float zz = 2.0f * r.z - 1.0f, zz2 = zz * zz;
        // z planes in mirror pairs (c, W-1-c), two weights per evaluation:
        // fewer live registers than all W at once
#pragma unroll
        for (int c2 = 0; c2 < (WZ + 1) / 2; ++c2) {
            float wlo = 1.0f, whi = 1.0f;
            if constexpr (DA == 3) wp.pair(zz, zz2, c2, wlo, whi);
#pragma unroll
            for (int h = 0; h < (DA == 3 ? 2 : 1); ++h) {
                const int c = h == 0 ? c2 : WZ - 1 - c2;
                const float wc = a * (h == 0 ? wlo : whi);
#pragma unroll
                for (int b = 0; b < WY; ++b) {
                    const float wbc = DA >= 2 ? wc * wy[b] : wc;
#pragma unroll
                    for (int i = 0; i < W; ++i) acc[c][b][i] = fmaf(wbc, wx[i], acc[c][b][i]);
                }
            }
        }
    }
    // the cell's total over its S splits, staged as stage[cell][c][b][i] by
    // the first lane of the cell; values go in groups of 8, each DPP step
    // over the group before the next, so no step waits on the one before
    float *accf = &acc[0][0][0];
    float *cst = stage + cell * VW;
    constexpr int G = 8;
#pragma unroll
    for (int k0 = 0; k0 < VW; k0 += G) {
        if constexpr (S == 4) {
#pragma unroll
            for (int k = k0; k < k0 + G && k < VW; ++k) accf[k] = quad_step1(accf[k]);
#pragma unroll
            for (int k = k0; k < k0 + G && k < VW; ++k) accf[k] = quad_step2(accf[k]);
        }
        if (split == 0) {
            if constexpr (VW % 4 == 0) {
#pragma unroll
                for (int k = k0; k < k0 + G && k < VW; k += 4)
                    *reinterpret_cast<float4 *>(cst + k) =
                        make_float4(accf[k], accf[k + 1], accf[k + 2], accf[k + 3]);
            } else {
#pragma unroll
                for (int k = k0; k < k0 + G && k < VW; ++k) cst[k] = accf[k];
            }
        }
    }
    __syncthreads();
    // region point (X, Y, Z) gets cell (dx, dy, dz)'s value at offset
    // (X - dx, Y - dy, Z - dz) when that offset lies in [0, W)
    float *out = static_cast<float *>(wi.priv) + (size_t)loc.lb * VOL;
    constexpr int KX = TILE < W ? TILE : W;  // loop over the shorter range
    for (int e = threadIdx.x; e < VOL; e += kBlock) {
        const int X = e % L;
        const int Y = DA >= 2 ? (e / L) % L : 0;
        const int Z = DA == 3 ? e / L2 : 0;
        float sum = 0.0f;
#pragma unroll 1
        for (int kz = 0; kz < (DA == 3 ? KX : 1); ++kz) {
            const int dz = DA == 3 ? (TILE <= W ? kz : Z - kz) : 0;
            const int oz = Z - dz;
            if (DA == 3 && (dz < 0 || dz >= TILE || oz < 0 || oz >= W)) continue;
            for (int ky = 0; ky < (DA >= 2 ? KX : 1); ++ky) {
                const int dy = DA >= 2 ? (TILE <= W ? ky : Y - ky) : 0;
                const int oy = Y - dy;
                if (DA >= 2 && (dy < 0 || dy >= TILE || oy < 0 || oy >= W)) continue;
#pragma unroll
                for (int kx = 0; kx < KX; ++kx) {
                    const int dx = TILE <= W ? kx : X - kx;
                    const int ox = X - dx;
                    if (dx < 0 || dx >= TILE || ox < 0 || ox >= W) continue;
                    const int cidx = (dz * (DA >= 2 ? TILE : 1) + dy) * TILE + dx;
                    sum += stage[cidx * VW + (oz * WY + oy) * W + ox];
                }
            }
        }
        out[e] = sum;
    }
}

template <int DA, int W, int TILE, int S>
__global__ __launch_bounds__(kBlock) void gather_cell_kernel(const WinInst *__restrict__ insts,
                                                             const int32_t *__restrict__ members,
                                                             const int32_t *__restrict__ prefix,
                                                             int cnt) {
    constexpr int m = W / 2;
    constexpr int L = TILE + W - 1;
    constexpr int L2 = DA >= 2 ? L * L : L;
    constexpr int VOL = DA == 3 ? L2 * L : L2;
    constexpr int CELLS = CellShape<DA, TILE>::cells;
    static_assert(CELLS * S == kBlock, "one thread per (cell, split)");
    constexpr int WY = DA >= 2 ? W : 1, WZ = DA == 3 ? W : 1;
    __shared__ float g_lds[VOL];
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    const NodeF32 *__restrict__ nodes = static_cast<const NodeF32 *>(wi.nodes);
    const float *__restrict__ grid = static_cast<const float *>(wi.grid);
    WinPoly<float, W> wp;
    wp.load(static_cast<const float *>(wi.poly));
    float *__restrict__ tmp = static_cast<float *>(wi.tmp);
    const int n = wi.n, tpd = wi.tpd;
    int tk, chunk, K;
    locate_chunk(wi.src_sub, wi.n_nonempty, wi.chunks, loc.lb, tk, chunk, K);
    const int tile_id = wi.tiles_ne[tk];
    const int key0 = tile_id * CELLS;
    const int ox = (tile_id % tpd) * TILE;
    const int oy = ((tile_id / tpd) % tpd) * TILE;
    const int oz = (tile_id / (tpd * tpd)) * TILE;
    const global_ptr<float> gg = as_global(static_cast<const float *>(grid));
    fill_lds<4, float>(
        VOL, kBlock,
        [&](int e) {
            size_t g = (size_t)wrap_index(ox - m + 1 + e % L, n);
            if constexpr (DA >= 2) g += (size_t)n * (size_t)wrap_index(oy - m + 1 + (e / L) % L, n);
            if constexpr (DA == 3) g += (size_t)n * (size_t)n * (size_t)wrap_index(oz - m + 1 + e / L2, n);
            return gg[g];
        },
        [&](int e, float v) { g_lds[e] = v; });
    __syncthreads();
    const int cell = threadIdx.x / S;
    int pb, pe;
    chunk_range(wi.cell_start[key0 + cell], wi.cell_start[key0 + cell + 1], chunk, K, pb, pe);
    const int lx = cell % TILE;
    const int ly = DA >= 2 ? (cell / TILE) % TILE : 0;
    const int lz = DA == 3 ? cell / (TILE * TILE) : 0;
    const int c0 = pb + (int)(threadIdx.x % S), c1 = pe;
    if (c0 >= c1) return;
    float g[WZ][WY][W];
#pragma unroll
    for (int c = 0; c < WZ; ++c)
#pragma unroll
        for (int b = 0; b < WY; ++b)
#pragma unroll
            for (int i = 0; i < W; ++i) g[c][b][i] = g_lds[((lz + c) * L + ly + b) * L + lx + i];
    // the next point's offsets and caller index load while the current one
    // is interpolated (no condition: past the end the last point again;
    // global views, so that nothing waits for them before their use)
    const global_ptr<float> nf = as_global(reinterpret_cast<const float *>(nodes));
    const global_ptr<int32_t> perm = as_global(wi.perm);
    float3 r_n = node_offsets(nf, c0);
    int q_n = perm[c0];
    for (int j = c0; j < c1; j += S) {
        const float3 r = r_n;
        const int q = q_n;
        r_n = node_offsets(nf, min(j + S, c1 - 1));
        q_n = perm[min(j + S, c1 - 1)];
        float wx[W], wy[W], wz[W];
        wp.eval(r.x, wx);
        if constexpr (DA >= 2) wp.eval(r.y, wy);
        if constexpr (DA == 3) wp.eval(r.z, wz);
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
        as_global_mut(tmp)[q] = acc;  // caller order
    }
}

// ------------------------------------------------------------------ per-cell, float64
// Float64 per-cell kernels (d_A = 3, W <= 6, tiles of 4^3 cells): a cell's
// W^3 float64 support does not fit one thread's registers, so the four
// lanes of a cell each own a quarter of it, (z half sz) x (y half sy) x all
// of x, and every lane of the cell walks all of its points, whose window
// weights the lane that loads each point evaluates once and stages in LDS
// (the window is even: offsets a and W-1-a come from one even/odd
// evaluation).  Spreading stages the cells' lower z halves in LDS, adds them
// into the region in a fixed order, then the upper halves; gathering adds
// the four lanes' partial interpolations with DPP quad steps.  No atomics:
// the results are the same bits for any scheduling.
__device__ __forceinline__ double dpp_f64(double v, int ctrl_is_xor1) {
    const long long b = __double_as_longlong(v);
    int lo, hi;
    if (ctrl_is_xor1) {
        lo = __builtin_amdgcn_mov_dpp((int)b, 0xB1, 0xF, 0xF, true);
        hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, true);
    } else {
        lo = __builtin_amdgcn_mov_dpp((int)b, 0x4E, 0xF, 0xF, true);
        hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x4E, 0xF, 0xF, true);
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Sum over the four lanes of a quad, the same bits in every lane.
__device__ __forceinline__ double quad_sum_f64(double v) {
    v = v + dpp_f64(v, 1);
    return v + dpp_f64(v, 0);
}

// Window weights of one point staged in LDS for the four lanes of its cell
// (float64 per-cell kernels): per axis all W weights by offset, from W/2
// even/odd evaluations (offsets a and W-1-a), then the coefficient
// (spreading) or the point's caller index (gathering).  The lane that loads
// a point evaluates them once; each lane then reads all of x and the y and
// z halves it owns.
template <int W>
struct Stage64 {
    static constexpr int H = W / 2;
    static constexpr int STRIDE = 3 * W + 2;  // doubles per point (even: 16-byte records)
    __device__ __forceinline__ static void put(const WinPoly<double, W, kPolyDegCell64> &wp,
                                               const double (&f)[3], double last, double *st) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const double z = 2.0 * f[t] - 1.0, z2 = z * z;
#pragma unroll
            for (int a = 0; a < H; ++a) {
                double lo, hi;
                wp.pair(z, z2, a, lo, hi);
                st[t * W + a] = lo;
                st[t * W + W - 1 - a] = hi;
            }
        }
        st[3 * W] = last;
    }
};

template <int W>
__global__ __launch_bounds__(kBlock, 2) void spread_cell64_kernel(const WinInst *__restrict__ insts,
                                                               const int32_t *__restrict__ members,
                                                               const int32_t *__restrict__ prefix,
                                                               int cnt) {
    constexpr int H = W / 2, TILE = 4, CELLS = 64;
    constexpr int L = TILE + W - 1, L2 = L * L, VOL = L2 * L;
    constexpr int VS = H * W * W;  // one z half of a cell's support
    constexpr int PER = (VOL + kBlock - 1) / kBlock;
    using ST = Stage64<W>;
    static_assert(W % 2 == 0 && W <= 6, "supports of 4 or 6 points");
    // the point loop stages weights here, the region formation the cells'
    // z halves afterwards
    constexpr int LDS_D = CELLS * VS > kBlock * ST::STRIDE ? CELLS * VS : kBlock * ST::STRIDE;
    __shared__ __align__(16) double lds[LDS_D];
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    const NodeF64 *__restrict__ nodes = static_cast<const NodeF64 *>(wi.nodes);
    const int32_t *__restrict__ perm = wi.perm;
    const double *__restrict__ alpha = wi.alpha;
    WinPoly<double, W, kPolyDegCell64> wp;
    wp.load(static_cast<const double *>(wi.poly));
    int tk, chunk, K;
    locate_chunk(wi.src_sub, wi.n_nonempty, wi.chunks, loc.lb, tk, chunk, K);
    const int key0 = wi.tiles_ne[tk] * CELLS;
    const int cell = threadIdx.x / 4, sub = threadIdx.x % 4;
    const int sz = sub >> 1, sy = sub & 1;
    int pb, pe;
    chunk_range(wi.cell_start[key0 + cell], wi.cell_start[key0 + cell + 1], chunk, K, pb, pe);
    // register (c, b, i) holds offset (sz H + c, sy H + b, i)
    double acc[H][H][W];
#pragma unroll
    for (int c = 0; c < H; ++c)
#pragma unroll
        for (int b = 0; b < H; ++b)
#pragma unroll
            for (int i = 0; i < W; ++i) acc[c][b][i] = 0.0;
    // the cell's points go through LDS in rounds of four, lane s of the
    // cell staging point s of a round (its record and coefficient loading a
    // round ahead); the lanes of a cell share a wave, whose LDS accesses
    // complete in order
    double *cst = lds + (threadIdx.x - sub) * ST::STRIDE;
    double nf[3] = {0.0, 0.0, 0.0}, na = 0.0;
    int jl = pb + sub;
    if (jl < pe) {
        const NodeF64 nd = nodes[jl];
        nf[0] = nd.f[0]; nf[1] = nd.f[1]; nf[2] = nd.f[2];
        na = alpha[perm[jl]];
    }
    for (int q0 = pb; q0 < pe; q0 += 4) {
        if (jl < pe) ST::put(wp, nf, na, cst + sub * ST::STRIDE);
        jl += 4;
        if (jl < pe) {
            const NodeF64 nd = nodes[jl];
            nf[0] = nd.f[0]; nf[1] = nd.f[1]; nf[2] = nd.f[2];
            na = alpha[perm[jl]];
        }
        const int kn = min(4, pe - q0);
        for (int k = 0; k < kn; ++k) {
            const double *ps = cst + k * ST::STRIDE;
            double wx[W], wy[H], wz[H];
#pragma unroll
            for (int i = 0; i < W; ++i) wx[i] = ps[i];
#pragma unroll
            for (int b = 0; b < H; ++b) wy[b] = ps[W + sy * H + b];
#pragma unroll
            for (int c = 0; c < H; ++c) wz[c] = ps[2 * W + sz * H + c];
            const double a = ps[3 * W];
#pragma unroll
            for (int c = 0; c < H; ++c) {
                const double wc = a * wz[c];
#pragma unroll
                for (int b = 0; b < H; ++b) {
                    const double wbc = wc * wy[b];
#pragma unroll
                    for (int i = 0; i < W; ++i) acc[c][b][i] = fma(wbc, wx[i], acc[c][b][i]);
                }
            }
        }
    }
    __syncthreads();  // every cell is done with its staged weights
    // the region: element (X, Y, Z) adds cell (dx, dy, dz)'s value at offset
    // (X - dx, Y - dy, Z - dz); lower z halves (offsets 0 .. H-1) first
    double *stage = lds;
    double sum[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) sum[k] = 0.0;
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
        if (half) __syncthreads();  // the first half's reads are done
        if (sz == half) {
            // stage[cell][c][oy][ox], c the plane inside the half
#pragma unroll
            for (int c = 0; c < H; ++c)
#pragma unroll
                for (int b = 0; b < H; ++b) {
                    double *row = stage + ((size_t)(cell * H + c) * W + sy * H + b) * W;
#pragma unroll
                    for (int i = 0; i < W; ++i) row[i] = acc[c][b][i];
                }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = threadIdx.x + k * kBlock;
            if (e >= VOL) break;
            const int X = e % L, Y = (e / L) % L, Z = e / L2;
            double s = sum[k];
            for (int dz = 0; dz < TILE; ++dz) {
                const int oz = Z - dz;
                if (oz < 0 || oz >= W) continue;
                if ((oz >= H) != (half == 1)) continue;
                const int c = oz - half * H;
                for (int dy = 0; dy < TILE; ++dy) {
                    const int oy = Y - dy;
                    if (oy < 0 || oy >= W) continue;
#pragma unroll
                    for (int dx = 0; dx < TILE; ++dx) {
                        const int ox = X - dx;
                        if (ox < 0 || ox >= W) continue;
                        const int cidx = (dz * TILE + dy) * TILE + dx;
                        s += stage[((size_t)(cidx * H + c) * W + oy) * W + ox];
                    }
                }
            }
            sum[k] = s;
        }
    }
    double *out = static_cast<double *>(wi.priv) + (size_t)loc.lb * VOL;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * kBlock;
        if (e < VOL) out[e] = sum[k];
    }
}

template <int W>
__global__ __launch_bounds__(kBlock, 2) void gather_cell64_kernel(const WinInst *__restrict__ insts,
                                                               const int32_t *__restrict__ members,
                                                               const int32_t *__restrict__ prefix,
                                                               int cnt) {
    constexpr int m = W / 2, H = W / 2, TILE = 4, CELLS = 64;
    constexpr int L = TILE + W - 1, L2 = L * L, VOL = L2 * L;
    using ST = Stage64<W>;
    __shared__ double g_lds[VOL];
    __shared__ __align__(16) double wst[kBlock * ST::STRIDE];
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    const NodeF64 *__restrict__ nodes = static_cast<const NodeF64 *>(wi.nodes);
    const double *__restrict__ grid = static_cast<const double *>(wi.grid);
    double *__restrict__ tmp = static_cast<double *>(wi.tmp);
    WinPoly<double, W, kPolyDegCell64> wp;
    wp.load(static_cast<const double *>(wi.poly));
    const int n = wi.n, tpd = wi.tpd;
    int tk, chunk, K;
    locate_chunk(wi.src_sub, wi.n_nonempty, wi.chunks, loc.lb, tk, chunk, K);
    const int tile_id = wi.tiles_ne[tk];
    const int key0 = tile_id * CELLS;
    const int ox = (tile_id % tpd) * TILE;
    const int oy = ((tile_id / tpd) % tpd) * TILE;
    const int oz = (tile_id / (tpd * tpd)) * TILE;
    const global_ptr<double> gg = as_global(static_cast<const double *>(grid));
    fill_lds<4, double>(
        VOL, kBlock,
        [&](int e) {
            size_t g = (size_t)wrap_index(ox - m + 1 + e % L, n);
            g += (size_t)n * (size_t)wrap_index(oy - m + 1 + (e / L) % L, n);
            g += (size_t)n * (size_t)n * (size_t)wrap_index(oz - m + 1 + e / L2, n);
            return gg[g];
        },
        [&](int e, double v) { g_lds[e] = v; });
    __syncthreads();
    const int cell = threadIdx.x / 4, sub = threadIdx.x % 4;
    const int sz = sub >> 1, sy = sub & 1;
    int pb, pe;
    chunk_range(wi.cell_start[key0 + cell], wi.cell_start[key0 + cell + 1], chunk, K, pb, pe);
    // the four lanes of a cell share its point count, so they leave together
    if (pb >= pe) return;
    const int lx = cell % TILE, ly = (cell / TILE) % TILE, lz = cell / (TILE * TILE);
    // register (c, b, i) holds offset (sz H + c, sy H + b, i)
    double g[H][H][W];
#pragma unroll
    for (int c = 0; c < H; ++c)
#pragma unroll
        for (int b = 0; b < H; ++b) {
            const double *row = g_lds + ((lz + sz * H + c) * L + ly + sy * H + b) * L + lx;
#pragma unroll
            for (int i = 0; i < W; ++i) g[c][b][i] = row[i];
        }
    // points through LDS in rounds of four, as in the spreading kernel (the
    // staged record ends with the point's caller index)
    const int32_t *__restrict__ perm = wi.perm;
    double *cst = wst + (threadIdx.x - sub) * ST::STRIDE;
    double nf[3] = {0.0, 0.0, 0.0};
    int np = 0;
    int jl = pb + sub;
    if (jl < pe) {
        const NodeF64 nd = nodes[jl];
        nf[0] = nd.f[0]; nf[1] = nd.f[1]; nf[2] = nd.f[2];
        np = perm[jl];
    }
    for (int q0 = pb; q0 < pe; q0 += 4) {
        if (jl < pe) ST::put(wp, nf, __longlong_as_double((long long)np), cst + sub * ST::STRIDE);
        jl += 4;
        if (jl < pe) {
            const NodeF64 nd = nodes[jl];
            nf[0] = nd.f[0]; nf[1] = nd.f[1]; nf[2] = nd.f[2];
            np = perm[jl];
        }
        const int kn = min(4, pe - q0);
        for (int k = 0; k < kn; ++k) {
            const double *ps = cst + k * ST::STRIDE;
            double wx[W], wy[H], wz[H];
#pragma unroll
            for (int i = 0; i < W; ++i) wx[i] = ps[i];
#pragma unroll
            for (int b = 0; b < H; ++b) wy[b] = ps[W + sy * H + b];
#pragma unroll
            for (int c = 0; c < H; ++c) wz[c] = ps[2 * W + sz * H + c];
            double part = 0.0;
#pragma unroll
            for (int c = 0; c < H; ++c) {
                double sc = 0.0;
#pragma unroll
                for (int b = 0; b < H; ++b) {
                    double sr = 0.0;
#pragma unroll
                    for (int i = 0; i < W; ++i) sr = fma(g[c][b][i], wx[i], sr);
                    sc = fma(sr, wy[b], sc);
                }
                part = fma(sc, wz[c], part);
            }
            const double v = quad_sum_f64(part);
            if (sub == 0) tmp[(int)__double_as_longlong(ps[3 * W])] = v;  // caller order
        }
    }
}

// ------------------------------------------------------------------ per-cell, wide supports
// Supports too wide for one thread's registers (d_A = 3, W = 8, float 32;
// 12-point supports go to the matrix-core kernels further down): SX x SY
// adjacent lanes of a cell each own one block of its support (half of the
// offsets along x and y, all of z), and every lane of the cell walks all of
// the cell's points.
//
// The window is even, so the polynomial of offset W-1-a at z = 2f-1 equals
// that of offset a at -z.  A lane owning the upper half of an axis indexes
// its offsets mirrored (register i holds offset W-1-i) and evaluates the
// lower-half polynomials at -z: every lane then evaluates the same W/2
// polynomials, whose coefficients sit in scalar registers.
//
// Such a lane holds up to 216 sums, so one workgroup of two waves takes a
// tile's 64 cells in groups, heaviest cells first; a wave's cells then hold
// about as many points each, and several workgroups share a compute unit,
// so one waiting for its fullest cell leaves the unit to the others.
// Spreading adds each cell's sums into the tile region with int64
// fixed-point LDS atomics at one scale per workgroup, fixed before the
// first point; gathering adds the block partials of a point over the
// cell's lanes in a fixed order.
template <int W> struct WideSplit;
// NPS / NPG: z passes of the spreading / gathering kernel
template <> struct WideSplit<8> { static constexpr int SX = 2, SY = 2, SZ = 1, NPS = 1, NPG = 1; };
constexpr int kWideTile = 4, kWideCells = 64, kWideThreads = 128;

template <int W>
constexpr int wide_lanes() { return WideSplit<W>::SX * WideSplit<W>::SY * WideSplit<W>::SZ; }
template <int W>
constexpr int wide_group_cells() { return kWideThreads / wide_lanes<W>(); }

// One axis of a lane's block: NA offsets, register i <-> support offset
// offset(s, i), weighted by a lower-half polynomial at z or -z.
template <int W, int SA>
struct WideAxis {
    static constexpr int NA = W / SA;
    // SA == 2: half s of the axis, mirrored when s == 1
    // SA == 1: the whole axis, lower half at z, upper half mirrored at -z
    __device__ __forceinline__ static int offset(int s, int i) {
        if constexpr (SA == 2) return s ? W - 1 - i : i;
        else return i;
    }
    __device__ __forceinline__ static void weights(const WinPoly<float, W> &hp, float z, int s,
                                                   float (&w)[NA]) {
        if constexpr (SA == 2) {
            const float zs = s ? -z : z;
#pragma unroll
            for (int i = 0; i < NA; ++i) w[i] = hp.at(zs, i);
        } else {
            const float z2 = z * z;
#pragma unroll
            for (int i = 0; i < W / 2; ++i) hp.pair(z, z2, i, w[i], w[W - 1 - i]);
        }
    }
    __device__ __forceinline__ static float weight(const WinPoly<float, W> &hp, float z, int s, int i) {
        if constexpr (SA == 2) return hp.at(s ? -z : z, i);
        else return i < W / 2 ? hp.at(z, i) : hp.at(-z, W - 1 - i);
    }
};

__device__ __forceinline__ float block_max_wide(float v, float *sh) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    float r = sh[0];
    for (int i = 1; i < kWideThreads / 64; ++i) r = fmaxf(r, sh[i]);
    return r;
}

// The chunk's share of each cell of the tile (first point, count) and the
// cells by count, heaviest first (ties by cell index).
struct WideCells {
    int pb[kWideCells], cnt[kWideCells], order[kWideCells];
};
__device__ __forceinline__ void wide_cells(const WinInst &wi, int key0, int chunk, int K,
                                           WideCells &cs) {
    const int t = threadIdx.x;
    if (t < kWideCells) {
        int pb, pe;
        chunk_range(wi.cell_start[key0 + t], wi.cell_start[key0 + t + 1], chunk, K, pb, pe);
        cs.pb[t] = pb;
        cs.cnt[t] = pe - pb;
    }
    __syncthreads();
    if (t < kWideCells) {
        const int c = cs.cnt[t];
        int r = 0;
        for (int u = 0; u < kWideCells; ++u) {
            const int cu = cs.cnt[u];
            r += (cu > c || (cu == c && u < t)) ? 1 : 0;
        }
        cs.order[r] = t;
    }
    __syncthreads();
}

// Window weights of one point staged in LDS for the lanes of its cell
// (gathering): per axis the lower-half polynomials at z (lo, offsets
// a < W/2) and at -z (hi, offset W-1-a), from one even/odd evaluation each,
// stored by offset (the hi half reversed, so that half s holds offsets
// s W/2 .. s W/2 + W/2 - 1 in order), then the point's caller index.  Each lane evaluates the weights of the
// point it loaded, so a point's polynomials are evaluated once instead of
// once per lane of the cell; a lane then reads the halves of each axis it
// owns.  (The spreading kernel keeps evaluating its own: there the staged
// weights' LDS and registers cost more occupancy than they save.)
template <int W>
struct WideStage {
    static constexpr int H = W / 2;
    static constexpr int STRIDE = 6 * H + 2;  // floats per point (even: float2 access)
    __device__ __forceinline__ static void put(const WinPoly<float, W> &hp, float4 p, float *st) {
        const float zs[3] = {2.0f * p.x - 1.0f, 2.0f * p.y - 1.0f, 2.0f * p.z - 1.0f};
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const float z = zs[t], z2 = z * z;
            float lo[H], hi[H];
#pragma unroll
            for (int a = 0; a < H; ++a) hp.pair(z, z2, a, lo[a], hi[a]);
#pragma unroll
            for (int a = 0; a < H; a += 2) {
                *reinterpret_cast<float2 *>(st + 2 * H * t + a) = make_float2(lo[a], lo[a + 1]);
                *reinterpret_cast<float2 *>(st + 2 * H * t + H + a) =
                    make_float2(hi[H - 1 - a], hi[H - 2 - a]);
            }
        }
        *reinterpret_cast<float2 *>(st + 6 * H) = make_float2(p.w, 0.0f);
    }
    // H weights of axis t, half s: offsets s H .. s H + H - 1
    __device__ __forceinline__ static void half(const float *st, int t, int s, float (&w)[H]) {
        const float *src = st + 2 * H * t + (s ? H : 0);
#pragma unroll
        for (int a = 0; a < H; a += 2) {
            const float2 v = *reinterpret_cast<const float2 *>(src + a);
            w[a] = v.x;
            w[a + 1] = v.y;
        }
    }
};

// A lane's block of the support (sx, sy, sz) and, for group g, its cell.
template <int W>
struct WideLane {
    int sub, sx, sy, sz;
    __device__ __forceinline__ WideLane() {
        constexpr int SY = WideSplit<W>::SY, SZ = WideSplit<W>::SZ;
        sub = (int)(threadIdx.x % wide_lanes<W>());
        sz = sub % SZ;
        sy = (sub / SZ) % SY;
        sx = sub / (SZ * SY);
    }
    // the two waves take the heavier half of a group in turn
    __device__ __forceinline__ int slot(int g) const {
        constexpr int CPG = wide_group_cells<W>();
        const int wave = (int)(threadIdx.x / 64);
        return g * CPG + ((wave + g) & 1) * (CPG / 2) + (int)(threadIdx.x % 64) / wide_lanes<W>();
    }
};

// x and y window weights of one point staged in LDS for the lanes of its
// cell (spreading): per axis the lower-half polynomials at z and at -z
// (offsets a and W-1-a), from one even/odd evaluation each, stored by
// offset (x then y, W each), the x weights already multiplied by the
// point's (scaled) coefficient.  A lane reads the half of each axis it
// owns; z weights, of which a lane needs only its z pass's planes, stay
// with each lane.
template <int W>
struct WideSpreadStage {
    static constexpr int H = W / 2;
    static constexpr int STRIDE = 4 * H;  // floats per point
    __device__ __forceinline__ static void put(const WinPoly<float, W> &hp, float4 p, float *st) {
        const float zs[2] = {2.0f * p.x - 1.0f, 2.0f * p.y - 1.0f};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const float z = zs[t], z2 = z * z;
            float lo[H], hi[H];
#pragma unroll
            for (int a = 0; a < H; ++a) {
                hp.pair(z, z2, a, lo[a], hi[a]);
                if (t == 0) {
                    lo[a] *= p.w;
                    hi[a] *= p.w;
                }
            }
#pragma unroll
            for (int a = 0; a < H; a += 2) {
                *reinterpret_cast<float2 *>(st + 2 * H * t + a) = make_float2(lo[a], lo[a + 1]);
                *reinterpret_cast<float2 *>(st + 2 * H * t + H + a) =
                    make_float2(hi[H - 1 - a], hi[H - 2 - a]);
            }
        }
    }
    // H weights of axis t (0: x, 1: y), half s: offsets s H .. s H + H - 1
    __device__ __forceinline__ static void half(const float *st, int t, int s, float (&w)[H]) {
        const float *src = st + 2 * H * t + (s ? H : 0);
#pragma unroll
        for (int a = 0; a < H; a += 2) {
            const float2 v = *reinterpret_cast<const float2 *>(src + a);
            w[a] = v.x;
            w[a + 1] = v.y;
        }
    }
};

template <int W>
__global__ __launch_bounds__(kWideThreads, 2) void spread_wide_kernel(
    const WinInst *__restrict__ insts, const int32_t *__restrict__ members,
    const int32_t *__restrict__ prefix, int cnt) {
    using SP = WideSplit<W>;
    using AZ = WideAxis<W, SP::SZ>;
    using ST = WideSpreadStage<W>;
    static_assert(SP::SX == 2 && SP::SY == 2, "x and y split in halves");
    constexpr int NT = kWideThreads, TPC = wide_lanes<W>();
    constexpr int NG = kWideCells / wide_group_cells<W>();
    constexpr int H = W / 2, PZ = AZ::NA / SP::NPS;
    constexpr int T = kWideTile, L = T + W - 1, VOL = L * L * L;
    __shared__ unsigned long long acc_lds[VOL];
    __shared__ __align__(16) float stage_xy[NT * ST::STRIDE];
    __shared__ float stage_z[NT];
    __shared__ WideCells cs;
    __shared__ float red[NT / 64];
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    const NodeF32 *__restrict__ nodes = static_cast<const NodeF32 *>(wi.nodes);
    const int32_t *__restrict__ perm = wi.perm;
    const double *__restrict__ alpha = wi.alpha;
    WinPoly<float, W> hp;
    hp.load(static_cast<const float *>(wi.poly));
    for (int e = threadIdx.x; e < VOL; e += NT) acc_lds[e] = 0ull;
    int tk, chunk, K;
    locate_chunk(wi.src_sub, wi.n_nonempty, wi.chunks, loc.lb, tk, chunk, K);
    const int key0 = wi.tiles_ne[tk] * kWideCells;
    wide_cells(wi, key0, chunk, K, cs);  // its barriers also order the zero fill
    // the scale, from the largest |coefficient| over the tile's points (a
    // superset of the chunk's) and the largest count of one cell: every
    // register sum of a cell then stays below 2^30 (weights are at most 1),
    // and an int64 region value adds at most one such sum per lane
    float amax = 0.0f;
    {
        const int t0 = wi.cell_start[key0], t1 = wi.cell_start[key0 + kWideCells];
        for (int j = t0 + (int)threadIdx.x; j < t1; j += 4 * NT) {
            int pi[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) pi[u] = j + u * NT < t1 ? perm[j + u * NT] : -1;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (pi[u] >= 0) amax = fmaxf(amax, abs_for_max(alpha[pi[u]]));
        }
    }
    amax = block_max_wide(amax, red);
    float *out = static_cast<float *>(wi.priv) + (size_t)loc.lb * VOL;
    if (!(amax > 0.0f && amax <= 3.0e38f)) {  // all zero, or not finite
        const float fill = amax > 0.0f ? NAN : 0.0f;
        for (int e = threadIdx.x; e < VOL; e += NT) out[e] = fill;
        return;
    }
    int ex2, ct;
    (void)frexpf(amax * 1.0000002f, &ex2);
    (void)frexpf(fmaxf((float)cs.cnt[cs.order[0]], 1.0f), &ct);
    const int Sx = 30 - ex2 - ct;
    const WideLane<W> ln;
    // this cell's staging slots: lane s of the cell stages point s of a round
    float *sxy = stage_xy + (threadIdx.x - ln.sub) * ST::STRIDE;
    float *sz = stage_z + (threadIdx.x - ln.sub);
#pragma unroll 1
    for (int g = 0; g < NG; ++g) {
        const int cell = cs.order[ln.slot(g)];
        const int pb = cs.pb[cell], pe = pb + cs.cnt[cell];
        if (pb >= pe) continue;  // the lanes of a cell go on together
        const int lx = cell % T, ly = (cell / T) % T, lz = cell / (T * T);
#pragma unroll  // constant pass: the polynomial index stays static
        for (int pass = 0; pass < SP::NPS; ++pass) {
            float acc[PZ][H][H];
#pragma unroll
            for (int c = 0; c < PZ; ++c)
#pragma unroll
                for (int b = 0; b < H; ++b)
#pragma unroll
                    for (int i = 0; i < H; ++i) acc[c][b][i] = 0.0f;
            // the cell's points go through LDS in rounds of TPC: lane s of
            // the cell stages the weights of point s of the round while the
            // next round's point loads, then every lane of the cell works
            // through the round's points; the lanes of a cell share a wave,
            // whose LDS accesses complete in order.  Coefficients carry the
            // fixed-point scale 2^Sx, so the sums are the region's integers
            // before truncation.
            float4 nx = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            int jl = pb + ln.sub;
            if (jl < pe) {
                const float3 r = node_offsets(nodes + jl);
                nx = make_float4(r.x, r.y, r.z, ldexpf((float)alpha[perm[jl]], Sx));
            }
            for (int q0 = pb; q0 < pe; q0 += TPC) {
                if (jl < pe) {
                    ST::put(hp, nx, sxy + ln.sub * ST::STRIDE);
                    sz[ln.sub] = 2.0f * nx.z - 1.0f;
                }
                jl += TPC;
                if (jl < pe) {
                    const float3 r = node_offsets(nodes + jl);
                    nx = make_float4(r.x, r.y, r.z, ldexpf((float)alpha[perm[jl]], Sx));
                }
                const int kn = min(TPC, pe - q0);
                for (int k = 0; k < kn; ++k) {
                    float wx[H], wy[H];
                    ST::half(sxy + k * ST::STRIDE, 0, ln.sx, wx);
                    ST::half(sxy + k * ST::STRIDE, 1, ln.sy, wy);
                    const float zz = sz[k];
                    static_assert(SP::SZ == 1 && SP::NPS == 1, "the whole z axis in one pass");
                    {
                        // the whole z axis: planes in mirror pairs
                        const float zz2 = zz * zz;
#pragma unroll
                        for (int c2 = 0; c2 < W / 2; ++c2) {
                            float wlo, whi;
                            hp.pair(zz, zz2, c2, wlo, whi);
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                const int c = h == 0 ? c2 : W - 1 - c2;
                                const float wc = h == 0 ? wlo : whi;
#pragma unroll
                                for (int b = 0; b < H; ++b) {
                                    const float wbc = wc * wy[b];
#pragma unroll
                                    for (int i = 0; i < H; ++i)
                                        acc[c][b][i] = fmaf(wbc, wx[i], acc[c][b][i]);
                                }
                            }
                        }
                    }
                }
            }
            // register sums into the region: |sum| < 2^30, truncated to an
            // integer (x and y offsets in order from the lane's half, z
            // mirrored for the upper half)
#pragma unroll
            for (int c = 0; c < PZ; ++c) {
                const int z = lz + AZ::offset(ln.sz, pass * PZ + c);
#pragma unroll
                for (int b = 0; b < H; ++b) {
                    unsigned long long *row =
                        acc_lds + (z * L + ly + ln.sy * H + b) * L + lx + ln.sx * H;
#pragma unroll
                    for (int i = 0; i < H; ++i)
                        atomicAdd(&row[i], (unsigned long long)(long long)(int)acc[c][b][i]);
                }
            }
        }
    }
    __syncthreads();
    const double inv = ldexp(1.0, -Sx);
    for (int e = threadIdx.x; e < VOL; e += NT) out[e] = (float)((double)(long long)acc_lds[e] * inv);
}

// Sum over the adjacent lanes of a cell, the same bits in every lane.
template <int TPC>
__device__ __forceinline__ float cell_lanes_sum(float v) {
    static_assert(TPC == 4 || TPC == 8, "4 or 8 lanes per cell");
    v = quad_step1(v);
    v = quad_step2(v);
    if constexpr (TPC == 8) v += __shfl_xor(v, 4, 64);
    return v;
}

// Row and plane strides of the grid tile in the gathering kernel's LDS.
template <int W>
struct WideGridPad {
    static constexpr int L = kWideTile + W - 1;
    static constexpr int RY = L;
    static constexpr int RZ = L * L;
};

template <int W>
__global__ __launch_bounds__(kWideThreads, 2) void gather_wide_kernel(
    const WinInst *__restrict__ insts, const int32_t *__restrict__ members,
    const int32_t *__restrict__ prefix, int cnt) {
    using SP = WideSplit<W>;
    using AX = WideAxis<W, SP::SX>;
    using AY = WideAxis<W, SP::SY>;
    using AZ = WideAxis<W, SP::SZ>;
    constexpr int NT = kWideThreads, TPC = wide_lanes<W>();
    constexpr int NG = kWideCells / wide_group_cells<W>();
    constexpr int WX = AX::NA, WY = AY::NA, PZ = AZ::NA / SP::NPG;
    constexpr int T = kWideTile, L = T + W - 1, L2 = L * L, VOL = L2 * L;
    constexpr int RY = WideGridPad<W>::RY, RZ = WideGridPad<W>::RZ;
    constexpr int m = W / 2;
    using ST = WideStage<W>;
    constexpr int H = ST::H;
    __shared__ float g_lds[RZ * L];
    __shared__ __align__(16) float wst[NT * ST::STRIDE];
    __shared__ float vsum[NT];  // a round's values, slot s of a cell for its point s
    __shared__ WideCells cs;
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    const NodeF32 *__restrict__ nodes = static_cast<const NodeF32 *>(wi.nodes);
    const float *__restrict__ grid = static_cast<const float *>(wi.grid);
    float *__restrict__ tmp = static_cast<float *>(wi.tmp);
    const int32_t *__restrict__ perm = wi.perm;
    WinPoly<float, W> hp;
    hp.load(static_cast<const float *>(wi.poly));
    const int n = wi.n, tpd = wi.tpd;
    int tk, chunk, K;
    locate_chunk(wi.src_sub, wi.n_nonempty, wi.chunks, loc.lb, tk, chunk, K);
    const int tile_id = wi.tiles_ne[tk];
    const int ox = (tile_id % tpd) * T;
    const int oy = ((tile_id / tpd) % tpd) * T;
    const int oz = (tile_id / (tpd * tpd)) * T;
    const global_ptr<float> gg = as_global(grid);
    fill_lds<4, float>(
        VOL, NT,
        [&](int e) {
            size_t gi = (size_t)wrap_index(ox - m + 1 + e % L, n);
            gi += (size_t)n * (size_t)wrap_index(oy - m + 1 + (e / L) % L, n);
            gi += (size_t)n * (size_t)n * (size_t)wrap_index(oz - m + 1 + e / L2, n);
            return gg[gi];
        },
        [&](int e, float v) { g_lds[(e / L2) * RZ + ((e / L) % L) * RY + e % L] = v; });
    wide_cells(wi, tile_id * kWideCells, chunk, K, cs);  // its barriers also order the fill
    const WideLane<W> ln;
    const bool lead = ln.sub == 0;
    const float *cst = wst + (threadIdx.x - ln.sub) * ST::STRIDE;  // the cell's points
    float *myst = wst + threadIdx.x * ST::STRIDE;
    float *cval = vsum + (threadIdx.x - ln.sub);
    static_assert(SP::SX == 2 && SP::SY == 2, "x and y split in halves");
#pragma unroll 1
    for (int g = 0; g < NG; ++g) {
        const int cell = cs.order[ln.slot(g)];
        const int pb = cs.pb[cell], pe = pb + cs.cnt[cell];
        if (pb >= pe) continue;  // the lanes of a cell go on together
        const int lx = cell % T, ly = (cell / T) % T, lz = cell / (T * T);
        // the cell's points go through LDS in rounds of TPC, lane s of the
        // cell staging point s of a round (offsets and caller index loading a
        // round ahead); within a round each pass loads its block of the
        // support and adds its part of the round's values, so a value is
        // written once, after the last pass
        float4 nx = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        int jl = pb + ln.sub;
        if (jl < pe) {
            const float3 r = node_offsets(nodes + jl);
            nx = make_float4(r.x, r.y, r.z, __int_as_float(perm[jl]));
        }
        for (int q0 = pb; q0 < pe; q0 += TPC) {
            ST::put(hp, nx, myst);
            jl += TPC;
            if (jl < pe) {
                const float3 r = node_offsets(nodes + jl);
                nx = make_float4(r.x, r.y, r.z, __int_as_float(perm[jl]));
            }
            const int kn = min(TPC, pe - q0);
#pragma unroll  // constant pass: the polynomial index stays static
            for (int pass = 0; pass < SP::NPG; ++pass) {
                // the lane's block, every axis in offset order from its half
                // (the staged weights are stored by offset)
                float gv[PZ][WY][WX];
#pragma unroll
                for (int c = 0; c < PZ; ++c) {
                    const int z = lz + ln.sz * (W / SP::SZ) + pass * PZ + c;
#pragma unroll
                    for (int b = 0; b < WY; ++b) {
                        const float *row = g_lds + z * RZ + (ly + ln.sy * H + b) * RY + lx + ln.sx * H;
#pragma unroll
                        for (int i = 0; i < WX; ++i) gv[c][b][i] = row[i];
                    }
                }
                for (int k = 0; k < kn; ++k) {
                    const float *ps = cst + k * ST::STRIDE;
                    float wx[WX], wy[WY];
                    ST::half(ps, 0, ln.sx, wx);
                    ST::half(ps, 1, ln.sy, wy);
                    float part = 0.0f;
                    auto plane = [&](int c) {
                        float sc = 0.0f;
#pragma unroll
                        for (int b = 0; b < WY; ++b) {
                            float sr = 0.0f;
#pragma unroll
                            for (int i = 0; i < WX; ++i) sr = fmaf(gv[c][b][i], wx[i], sr);
                            sc = fmaf(sr, wy[b], sc);
                        }
                        return sc;
                    };
                    static_assert(SP::SZ == 1 && SP::NPG == 1, "the whole z axis in one pass");
                    {
                        float zlo[H], zhi[H];
                        ST::half(ps, 2, 0, zlo);
                        ST::half(ps, 2, 1, zhi);
#pragma unroll
                        for (int c = 0; c < H; ++c) part = fmaf(plane(c), zlo[c], part);
#pragma unroll
                        for (int c = 0; c < H; ++c) part = fmaf(plane(H + c), zhi[c], part);
                    }
                    const float v = cell_lanes_sum<TPC>(part);
                    if (lead) cval[k] = pass == 0 ? v : cval[k] + v;
                }
            }
            // lane s of the cell writes the value of the point it staged
            if (ln.sub < kn) tmp[__float_as_int(myst[6 * H])] = cval[ln.sub];  // caller order
        }
    }
}

// ------------------------------------------------------------------ per-tile, matrix cores
// 12-point supports in 3-D.  A tile of 4^3 cells has a 15^3 region, which
// pads to 15 planes of 16 x 16.  Spreading adds, for each plane z,
//   R_z[y][x] += sum_j (a_j wz_j[z] wy_j[y]) wx_j[x]
// over the tile's points j, each point's weights placed at its cell's offset
// in zero-padded 16-vectors: a (16 x K) by (K x 16) product for K points,
// four points per V_MFMA_F32_16X16X4_F32.  Gathering contracts the other
// way: T_z[y][j] = sum_x G_z[y][x] wx_j[x] by the same instruction with x as
// the inner dimension, then v_j = sum_z wz_j[z] sum_y wy_j[y] T_z[y][j] on
// the vector units.  Instruction layout (one 16 x 16 block, inner dimension
// 4): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16], and its four
// result registers hold D[4 (l / 16) + r][l % 16].
//
// One lane evaluates a point's weights and stages them in LDS for its wave
// (each axis's W weights and the point's cell offsets in the tile); a lane
// of the instruction reads the weight at its own row or column, which is
// zero outside the point's support.  A tile's points are sorted by cell, z
// slowest, so a run of them mostly shares one z layer and touches W of the
// 15 planes.  Compared with the per-cell kernels there are no atomics: a
// wave's sums stay in its result registers until the end, where the four
// waves' regions are added in a fixed order.
constexpr int kMfmaThreads = 256, kMfmaRound = 64;  // points a wave stages at once
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <int W>
struct MfmaRegion {
    static constexpr int L = kWideTile + W - 1;  // region edge
    static_assert(L <= 16, "region rows and columns fit one 16-wide block");
    static_assert(W <= 12, "z weights take 12 staged slots");
    static_assert(L - W == 3, "four z layers of cells per tile");
};

// Staging of one point: the W weights of each axis (z, then x, then y
// multiplied by ya), then the cell offsets lx | ly << 8; a lane applies the
// offsets when it reads.  An odd stride keeps the lanes' staging writes in
// different LDS banks.
constexpr int kSpreadStride = 37;
template <int W>
__device__ __forceinline__ void mfma_stage_compact(const WinPoly<float, W> &hp, float3 r, int lx, int ly,
                                                   float ya, float *st) {
    static_assert(3 * W + 1 <= kSpreadStride, "a point's weights fit its slot");
    float w[W];
    hp.eval(r.z, w);
#pragma unroll
    for (int a = 0; a < W; ++a) st[a] = w[a];
    hp.eval(r.x, w);
#pragma unroll
    for (int a = 0; a < W; ++a) st[W + a] = w[a];
    hp.eval(r.y, w);
#pragma unroll
    for (int a = 0; a < W; ++a) st[2 * W + a] = ya * w[a];
    st[3 * W] = __int_as_float(lx | ly << 8);
}

// LDS written by one lane of a wave and then read by others: LDS operations
// of a wave complete in order; this keeps the compiler from moving them.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Planes [zlo, zhi) of a step: W planes from a constant first one when the
// step's points share a z layer, else all of them.  f(Z0, NZ) runs planes
// Z0 .. Z0 + NZ - 1 with both constant, so the per-plane registers stay
// statically indexed.
template <int W, typename F>
__device__ __forceinline__ void mfma_planes(int zlo, int zhi, F &&f) {
    constexpr int L = MfmaRegion<W>::L;
    using std::integral_constant;
    if (zhi - zlo == W) {
        switch (zlo) {
            case 0: f(integral_constant<int, 0>{}, integral_constant<int, W>{}); return;
            case 1: f(integral_constant<int, 1>{}, integral_constant<int, W>{}); return;
            case 2: f(integral_constant<int, 2>{}, integral_constant<int, W>{}); return;
            case 3: f(integral_constant<int, 3>{}, integral_constant<int, W>{}); return;
            default: break;
        }
    }
    f(integral_constant<int, 0>{}, integral_constant<int, L>{});
}

// The workgroup's tile (origin cell) and its points: a contiguous share of
// the tile's sorted points, chunk `chunk` of K.
struct MfmaTile {
    int ox, oy, oz, c0, c1;
    int key0, chunk, K;  // first (tile, cell) key; chunk `chunk` of K
};
__device__ __forceinline__ MfmaTile mfma_tile(const WinInst &wi, int lb) {
    int tk, chunk, K;
    locate_chunk(wi.src_sub, wi.n_nonempty, wi.chunks, lb, tk, chunk, K);
    const int tile_id = wi.tiles_ne[tk], tpd = wi.tpd;
    MfmaTile t;
    t.ox = (tile_id % tpd) * kWideTile;
    t.oy = ((tile_id / tpd) % tpd) * kWideTile;
    t.oz = (tile_id / (tpd * tpd)) * kWideTile;
    t.key0 = tile_id * kWideCells;
    t.chunk = chunk;
    t.K = K;
    chunk_range(wi.cell_start[t.key0], wi.cell_start[t.key0 + kWideCells], chunk, K, t.c0, t.c1);
    return t;
}

// Wave wv's share of the workgroup's points: whole steps of S points, the
// workgroup's steps split evenly over its waves (only its last step short).
__device__ __forceinline__ void mfma_wave_share(const MfmaTile &t, int wv, int S, int &q0, int &q1) {
    constexpr int NWV = kMfmaThreads / 64;
    const int steps = (t.c1 - t.c0 + S - 1) / S;
    q0 = min(t.c1, t.c0 + S * (steps * wv / NWV));
    q1 = min(t.c1, t.c0 + S * (steps * (wv + 1) / NWV));
}

// Spreading: wave wv takes the points of the tile's cell layer wv (cells
// 16 wv .. 16 wv + 15, their chunk's share), whose z supports all start at
// plane wv, so its steps touch W planes at constant indices.
template <int W>
__global__ __launch_bounds__(kMfmaThreads) void spread_mfma_kernel(
    const WinInst *__restrict__ insts, const int32_t *__restrict__ members,
    const int32_t *__restrict__ prefix, int cnt) {
    constexpr int L = MfmaRegion<W>::L, VOL = L * L * L, NWV = kMfmaThreads / 64;
    constexpr int LAYER = kWideTile * kWideTile;  // cells per z layer
    constexpr int FR = 17, FP = 16 * FR;  // row and plane strides of the summed regions
    constexpr int STAGE = NWV * kMfmaRound * kSpreadStride, PLANES = 2 * L * FP;
    static_assert(NWV == kWideTile, "one wave per cell layer");
    __shared__ __align__(16) float lds[STAGE > PLANES ? STAGE : PLANES];
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    const NodeF32 *__restrict__ nodes = static_cast<const NodeF32 *>(wi.nodes);
    const int32_t *__restrict__ perm = wi.perm;
    const double *__restrict__ alpha = wi.alpha;
    WinPoly<float, W> hp;
    hp.load(static_cast<const float *>(wi.poly));
    const MfmaTile tl = mfma_tile(wi, loc.lb);
    const int lane = (int)threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int g = lane >> 4, col = lane & 15;
    int q0, q1;
    chunk_range(wi.cell_start[tl.key0 + LAYER * wv], wi.cell_start[tl.key0 + LAYER * (wv + 1)],
                tl.chunk, tl.K, q0, q1);
    float *wst = lds + wv * (kMfmaRound * kSpreadStride);
    mfma_f4 acc[L];
#pragma unroll
    for (int c = 0; c < L; ++c) acc[c] = mfma_f4{0.0f, 0.0f, 0.0f, 0.0f};
    auto run = [&](auto z0c) {
        constexpr int Z0 = decltype(z0c)::value;
        for (int base = q0; base < q1; base += kMfmaRound) {
            const int kn = min(kMfmaRound, q1 - base);
            float *st = wst + lane * kSpreadStride;
            wave_lds_sync();  // the previous round's reads come first
            if (lane < kn) {
                const int j = base + lane;
                const float4 nd = *reinterpret_cast<const float4 *>(nodes + j);
                const uint32_t cb = __float_as_uint(nd.w);
                const int lx = (int)(cb & 1023u) - tl.ox, ly = (int)((cb >> 10) & 1023u) - tl.oy;
                mfma_stage_compact(hp, make_float3(nd.x, nd.y, nd.z), lx, ly, (float)alpha[perm[j]], st);
            } else {
#pragma unroll
                for (int q = 0; q < 3 * W + 1; ++q) st[q] = 0.0f;  // a step's missing points add zero
            }
            wave_lds_sync();
            for (int k0 = 0; k0 < kn; k0 += 4) {
                // lanes of group g hold the step's point g: A column g (row
                // y = col), B row g (column x = col), each the point's weight
                // at that offset from its cell, zero outside the support
                const float *sp = wst + (k0 + g) * kSpreadStride;
                const int lxy = __float_as_int(sp[3 * W]);
                const int dx = col - (lxy & 255), dy = col - (lxy >> 8);
                const float wxv = sp[W + min(max(dx, 0), W - 1)];
                const float wyv = sp[2 * W + min(max(dy, 0), W - 1)];
                const float xb = (unsigned)dx < (unsigned)W ? wxv : 0.0f;
                const float ya = (unsigned)dy < (unsigned)W ? wyv : 0.0f;
#pragma unroll
                for (int c = Z0; c < Z0 + W; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya * sp[c - Z0], xb, acc[c], 0, 0, 0);
            }
        }
    };
    switch (wv) {
        case 0: run(std::integral_constant<int, 0>{}); break;
        case 1: run(std::integral_constant<int, 1>{}); break;
        case 2: run(std::integral_constant<int, 2>{}); break;
        default: run(std::integral_constant<int, 3>{}); break;
    }
    // the four waves' regions: (0 + 2) + (1 + 3), in a padded layout whose
    // rows are FR floats apart (a wave's four row groups then write to
    // different LDS banks)
    __syncthreads();
    if (wv < 2) {
        float *dst = lds + wv * (L * FP);
#pragma unroll
        for (int c = 0; c < L; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[c * FP + (4 * g + r) * FR + col] = acc[c][r];
    }
    __syncthreads();
    if (wv >= 2) {
        float *dst = lds + (wv - 2) * (L * FP);
#pragma unroll
        for (int c = 0; c < L; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[c * FP + (4 * g + r) * FR + col] += acc[c][r];
    }
    __syncthreads();
    float *out = static_cast<float *>(wi.priv) + (size_t)loc.lb * VOL;
    for (int e = threadIdx.x; e < VOL; e += kMfmaThreads) {
        const int i = (e / (L * L)) * FP + ((e / L) % L) * FR + e % L;
        out[e] = lds[i] + lds[L * FP + i];
    }
}

// Gathering stages each point the same way, with lz << 16 added to the cell
// offsets and the caller's index after them.
constexpr int kGatherStride = 39;

template <int W>
__global__ __launch_bounds__(kMfmaThreads) __attribute__((amdgpu_waves_per_eu(4))) void gather_mfma_kernel(
    const WinInst *__restrict__ insts, const int32_t *__restrict__ members,
    const int32_t *__restrict__ prefix, int cnt) {
    constexpr int L = MfmaRegion<W>::L, NWV = kMfmaThreads / 64, m = W / 2;
    constexpr int RS = 20, PS = 16 * RS;  // LDS row and plane strides of the region
    constexpr int STAGE = NWV * kMfmaRound * kGatherStride, PLANES = L * PS;
    static_assert(3 * W + 2 <= kGatherStride, "a point's record fits its slot");
    __shared__ __align__(16) float lds[STAGE > PLANES ? STAGE : PLANES];
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    const NodeF32 *__restrict__ nodes = static_cast<const NodeF32 *>(wi.nodes);
    const float *__restrict__ grid = static_cast<const float *>(wi.grid);
    float *__restrict__ tmp = static_cast<float *>(wi.tmp);
    const int32_t *__restrict__ perm = wi.perm;
    WinPoly<float, W> hp;
    hp.load(static_cast<const float *>(wi.poly));
    const MfmaTile tl = mfma_tile(wi, loc.lb);
    const int n = wi.n;
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    const int g = lane >> 4, col = lane & 15;
    // the tile's region of the grid, padded to 16 x 16 planes with zeros
    // (rows RS apart: the lanes' row reads below then meet fewer LDS banks):
    // thread (x, y) loads its column's L planes at once
    {
        static_assert(kMfmaThreads == 256, "one thread per (x, y) of a plane");
        const int x = (int)threadIdx.x & 15, y = (int)threadIdx.x >> 4;
        const bool in = x < L && y < L;
        const global_ptr<float> gxy =
            as_global(grid) + (size_t)wrap_index(tl.ox - m + 1 + min(x, L - 1), n) +
            (size_t)n * (size_t)wrap_index(tl.oy - m + 1 + min(y, L - 1), n);
        float v[L];
#pragma unroll
        for (int z = 0; z < L; ++z) v[z] = gxy[(size_t)n * (size_t)n * (size_t)wrap_index(tl.oz - m + 1 + z, n)];
#pragma unroll
        for (int z = 0; z < L; ++z) lds[z * PS + y * RS + x] = in ? v[z] : 0.0f;
    }
    __syncthreads();
    // A operand of every plane, kept in registers: row col, x = 4 g .. 4 g + 3
    // (step s of a plane's four takes x = 4 (l / 16) + s in lane l)
    float4 gv[L];
#pragma unroll
    for (int c = 0; c < L; ++c) gv[c] = *reinterpret_cast<const float4 *>(lds + c * PS + col * RS + 4 * g);
    __syncthreads();  // the region's LDS becomes staging space
    int q0, q1;
    mfma_wave_share(tl, wv, 16, q0, q1);
    float *wst = lds + wv * (kMfmaRound * kGatherStride);
    for (int base = q0; base < q1; base += kMfmaRound) {
        const int kn = min(kMfmaRound, q1 - base);
        float *st = wst + lane * kGatherStride;
        wave_lds_sync();
        if (lane < kn) {
            const int j = base + lane;
            const float4 nd = *reinterpret_cast<const float4 *>(nodes + j);
            const uint32_t cb = __float_as_uint(nd.w);
            const int lx = (int)(cb & 1023u) - tl.ox, ly = (int)((cb >> 10) & 1023u) - tl.oy;
            const int lz = (int)((cb >> 20) & 1023u) - tl.oz;
            mfma_stage_compact(hp, make_float3(nd.x, nd.y, nd.z), lx, ly | lz << 8, 1.0f, st);
            st[3 * W + 1] = __int_as_float(perm[j]);
        } else {
#pragma unroll
            for (int q = 0; q < 3 * W + 1; ++q) st[q] = 0.0f;  // reads zero weights
        }
        wave_lds_sync();
        for (int kb = 0; kb < kn; kb += 16) {
            // lane l takes point kb + l % 16 (B column and result column):
            // its x weights at x = 4 g + s and y weights at rows 4 g + r,
            // each at that offset from its cell, zero outside the support
            const int p = kb + col;
            const float *sp = wst + p * kGatherStride;
            const int lxyz = __float_as_int(sp[3 * W]);
            const int lx = lxyz & 255, ly = (lxyz >> 8) & 255, lzp = lxyz >> 16;
            float xs[4], ys[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int dx = 4 * g + s - lx, dy = 4 * g + s - ly;
                const float wxv = sp[W + min(max(dx, 0), W - 1)];
                const float wyv = sp[2 * W + min(max(dy, 0), W - 1)];
                xs[s] = (unsigned)dx < (unsigned)W ? wxv : 0.0f;
                ys[s] = (unsigned)dy < (unsigned)W ? wyv : 0.0f;
            }
            // the block's planes: its points are sorted by z layer
            const int zlo = __builtin_amdgcn_readfirstlane(__float_as_int(wst[kb * kGatherStride + 3 * W]) >> 16);
            const int zhi = __builtin_amdgcn_readfirstlane(
                                __float_as_int(wst[min(kb + 15, kn - 1) * kGatherStride + 3 * W]) >> 16) + W;
            float part = 0.0f;
            mfma_planes<W>(zlo, zhi, [&](auto z0c, auto nzc) {
                constexpr int Z0 = decltype(z0c)::value, NZ = decltype(nzc)::value;
#pragma unroll
                for (int c = Z0; c < Z0 + NZ; ++c) {
                    mfma_f4 t = {0.0f, 0.0f, 0.0f, 0.0f};
                    t = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[c].x, xs[0], t, 0, 0, 0);
                    t = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[c].y, xs[1], t, 0, 0, 0);
                    t = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[c].z, xs[2], t, 0, 0, 0);
                    t = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[c].w, xs[3], t, 0, 0, 0);
                    // rows 4 g + r of the plane, weighted by y, then by z
                    const float s = fmaf(ys[0], t[0], fmaf(ys[1], t[1], fmaf(ys[2], t[2], ys[3] * t[3])));
                    float wz;
                    if constexpr (NZ == W) {
                        wz = sp[c - Z0];
                    } else {
                        const int d = c - lzp;
                        const float v = sp[min(max(d, 0), W - 1)];
                        wz = (unsigned)d < (unsigned)W ? v : 0.0f;
                    }
                    part = fmaf(wz, s, part);
                }
            });
            // the four row groups of the point, in the same order in every lane
            part += __shfl_xor(part, 16, 64);
            part += __shfl_xor(part, 32, 64);
            if (g == 0 && p < kn) tmp[__float_as_int(sp[3 * W + 1])] = part;  // caller order
        }
    }
}

// ------------------------------------------------------------------ gather, per point
template <typename T, int DA, int W>
__global__ __launch_bounds__(kBlock) void gather_pt_kernel(const WinInst *__restrict__ insts,
                                                           const int32_t *__restrict__ members,
                                                           const int32_t *__restrict__ prefix,
                                                           int cnt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *lds = reinterpret_cast<T *>(smem_raw);
    constexpr int m = W / 2;
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    using Node = typename NodeOf<T>::type;
    const Node *__restrict__ nodes = static_cast<const Node *>(wi.nodes);
    const T *__restrict__ grid = static_cast<const T *>(wi.grid);
    const T *__restrict__ poly = static_cast<const T *>(wi.poly);
    T *__restrict__ tmp = static_cast<T *>(wi.tmp);
    const int tile = wi.tile, tpd = wi.tpd, n = wi.n;
    const int L = tile + W - 1;
    const int L2 = DA >= 2 ? L * L : L;
    const int vol = DA == 3 ? L2 * L : L2;
    const SubProblem sp = wi.subs[loc.lb];
    const int ox = (sp.tile % tpd) * tile;
    const int oy = ((sp.tile / tpd) % tpd) * tile;
    const int oz = (sp.tile / (tpd * tpd)) * tile;
    for (int e = threadIdx.x; e < vol; e += kBlock) {
        const int ex = e % L;
        size_t g = (size_t)wrap_index(ox - m + 1 + ex, n);
        if constexpr (DA >= 2) g += (size_t)n * (size_t)wrap_index(oy - m + 1 + (e / L) % L, n);
        if constexpr (DA == 3) g += (size_t)n * (size_t)n * (size_t)wrap_index(oz - m + 1 + e / L2, n);
        lds[e] = grid[g];
    }
    __syncthreads();
    const int end = sp.start + sp.count;
    for (int j = sp.start + threadIdx.x; j < end; j += kBlock) {
        const Node rec = nodes[j];
        const int lx = int(rec.cell & 1023u) - ox;
        T wx[W];
        window_weights<T, W>(poly, rec.f[0], wx);
        T acc = T(0);
        if constexpr (DA == 1) {
#pragma unroll
            for (int i = 0; i < W; ++i) acc += lds[lx + i] * wx[i];
        } else {
            const int ly = int((rec.cell >> 10) & 1023u) - oy;
            T wy[W];
            window_weights<T, W>(poly, rec.f[1], wy);
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
                window_weights<T, W>(poly, rec.f[2], wz);
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
        tmp[wi.perm[j]] = acc;  // caller order
    }
}

// ------------------------------------------------------------------ permute
// The window's coefficients in its sorted point order, as[j] = alpha[perm[j]],
// written to the instance's value buffer (the gather overwrites it later);
// per-point windows only (the per-cell spread reads alpha[perm[j]] itself).
// Blocks: ceil(N / (4 kBlock)) per instance.
// Elements per thread of the permutation and combine kernels: their loads
// land at random positions, so each thread first issues all its index loads,
// then all its gathers, keeping several misses in flight.
constexpr int kPermutePerThread = 8;
constexpr int kPermuteSpan = kPermutePerThread * kBlock;

template <typename T>
__global__ __launch_bounds__(kBlock) void permute_kernel(const WinInst *__restrict__ insts,
                                                         const int32_t *__restrict__ members,
                                                         const int32_t *__restrict__ prefix,
                                                         int cnt) {
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    const int32_t *__restrict__ perm = wi.perm;
    const double *__restrict__ alpha = wi.alpha;
    T *__restrict__ as = static_cast<T *>(wi.tmp);
    const int j0 = loc.lb * kPermuteSpan + threadIdx.x;
    int idx[kPermutePerThread];
    double v[kPermutePerThread];
#pragma unroll
    for (int e = 0; e < kPermutePerThread; ++e) {
        const int j = j0 + e * kBlock;
        idx[e] = j < wi.N ? perm[j] : -1;
    }
#pragma unroll
    for (int e = 0; e < kPermutePerThread; ++e) v[e] = idx[e] >= 0 ? alpha[idx[e]] : 0.0;
#pragma unroll
    for (int e = 0; e < kPermutePerThread; ++e) {
        const int j = j0 + e * kBlock;
        if (j < wi.N) as[j] = static_cast<T>(v[e]);
    }
}

// ------------------------------------------------------------------ tile sum
// Regions of the same tile (several sub-problems or chunks) are added
// elementwise, in region order, into one region per non-empty tile:
// src_sub[k] .. src_sub[k+1]-1 are the regions of the k-th non-empty tile.
// Blocks: non-empty tiles x ceil(vol / kBlock).
template <typename T>
__global__ __launch_bounds__(kBlock) void tile_sum_kernel(const WinInst *__restrict__ insts,
                                                          const int32_t *__restrict__ members,
                                                          const int32_t *__restrict__ prefix,
                                                          int cnt) {
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    const int vol = wi.vol;
    const int per = (vol + kBlock - 1) / kBlock;
    const int k = loc.lb / per;
    const int e = (loc.lb % per) * kBlock + threadIdx.x;
    if (e >= vol) return;
    const global_ptr<T> priv = as_global(static_cast<const T *>(wi.priv));
    // the tile's regions (per-cell windows: chunks k K .. k K + K - 1, no load)
    const int s0 = wi.chunks > 0 ? k * wi.chunks : wi.src_sub[k];
    const int s1 = wi.chunks > 0 ? s0 + wi.chunks : wi.src_sub[k + 1];
    // regions in order, their loads issued eight at a time (a missing one as +0)
    constexpr int B = 8;
    double s = 0.0;
    for (int q = s0; q < s1; q += B) {
        T v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) v[u] = load_or_zero(priv + ((size_t)(q + u) * vol + e), q + u < s1);
#pragma unroll
        for (int u = 0; u < B; ++u) s += (double)v[u];
    }
    static_cast<T *>(wi.treg)[(size_t)k * vol + e] = static_cast<T>(s);
}

// ------------------------------------------------------------------ fold
// One workgroup per destination tile: every grid point of the tile is the
// sum, in the fixed order of the plan's pair list, of the region values of
// the non-empty tiles whose region covers it (regions wrap periodically: per
// dimension the region indices of grid point o + c are the values in [0, L)
// congruent to b + c mod n, b the tile origin's offset in the region).
// Writes every grid point, so no zero fill is needed.
constexpr int kFoldBatch = 16;  // region reads in flight per thread
constexpr int kFoldZeroPasses = 4;  // zeroing workgroups: passes of the threads over tiles
constexpr int kFoldPairsLds = 512;  // a tile's pair list staged in LDS up to this length

// One workgroup per tile that receives regions, in the plan's order
// (entries -1 are padding).  A small tile's cells get S threads each:
// thread s of a cell adds regions s, s + S, s + 2S, ... of the tile's list,
// and the S partial sums are then added in order of s.  The tile's pair
// list goes to LDS first (when it fits), so that the region reads of a
// thread depend on no other global load and go out kFoldBatch at a time.
// The remaining workgroups zero the tiles that receive no region,
// kFoldZeroPasses passes of the threads over tiles each.
template <typename T, int DA>
__global__ __launch_bounds__(kBlock) void fold_kernel(const WinInst *__restrict__ insts,
                                                      const int32_t *__restrict__ members,
                                                      const int32_t *__restrict__ prefix,
                                                      int cnt) {
    __shared__ double part[kBlock];
    __shared__ int2 pairs_lds[kFoldPairsLds];
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    const global_ptr<T> src =
        as_global(static_cast<const T *>(wi.n_regions != wi.n_nonempty ? wi.treg : wi.priv));
    T *__restrict__ grid = static_cast<T *>(wi.grid);
    const int n = wi.n, tile = wi.tile, tpd = wi.tpd, vol = wi.vol;
    const int L = tile + wi.width - 1;
    const int L2 = DA >= 2 ? L * L : L;
    int cells = tile;
    if (DA >= 2) cells *= tile;
    if (DA == 3) cells *= tile;
    auto grid_index = [&](int d, int c) {
        size_t g = (size_t)((d % tpd) * tile + c % tile);
        if (DA >= 2) g += (size_t)n * (size_t)(((d / tpd) % tpd) * tile + (c / tile) % tile);
        if (DA == 3)
            g += (size_t)n * (size_t)n * (size_t)((d / (tpd * tpd)) * tile + c / (tile * tile));
        return g;
    };
    if (loc.lb >= wi.fold_act) {
        const int per = cells >= kBlock ? 1 : kBlock / cells;  // tiles per pass of the threads
        const int first = wi.fold_act + (loc.lb - wi.fold_act) * per * kFoldZeroPasses;
        const int last = min(first + per * kFoldZeroPasses, wi.fold_len);
        const int c0 = cells >= kBlock ? (int)threadIdx.x : (int)threadIdx.x % cells;
        const int cstep = cells >= kBlock ? kBlock : cells;
        for (int e = first + (cells >= kBlock ? 0 : (int)threadIdx.x / cells); e < last; e += per) {
            const int dz = wi.fold_tiles[e];
            for (int c = c0; c < cells; c += cstep) grid[grid_index(dz, c)] = T(0);
        }
        return;
    }
    const int d = wi.fold_tiles[loc.lb];
    if (d < 0) return;  // padding (the whole workgroup)
    const int p0 = wi.fold_start[d], p1 = wi.fold_start[d + 1];
    const bool staged = p1 - p0 <= kFoldPairsLds;
    if (staged) {
        for (int e = (int)threadIdx.x; e < p1 - p0; e += kBlock) pairs_lds[e] = wi.fold_pairs[p0 + e];
        __syncthreads();
    }
    auto pair_at = [&](int q) { return staged ? pairs_lds[q - p0] : wi.fold_pairs[q]; };
    const global_ptr<long long> fpairs = as_global(reinterpret_cast<const long long *>(wi.fold_pairs));
    // sum over regions first, first + stride, ... of cell c
    auto cell_sum = [&](int c, int first, int stride) {
        const int cx = c % tile;
        const int cy = DA >= 2 ? (c / tile) % tile : 0;
        const int cz = DA == 3 ? c / (tile * tile) : 0;
        double s = 0.0;
        if (L <= n) {
            // each region element lands on one grid point: at most one read
            // per region; kFoldBatch regions' reads in flight, added in order
            for (int p = first; p < p1; p += kFoldBatch * stride) {
                // the batch's pairs first (from LDS, or from global memory
                // when the list did not fit): waiting for them then waits
                // for no region read, and the region reads go out together
                int2 prs[kFoldBatch];
                if (staged) {
#pragma unroll
                    for (int u = 0; u < kFoldBatch; ++u) prs[u] = pairs_lds[min(p + u * stride, p1 - 1) - p0];
                } else {
#pragma unroll
                    for (int u = 0; u < kFoldBatch; ++u) {
                        const long long w = fpairs[min(p + u * stride, p1 - 1)];  // {x, y}, x low
                        prs[u] = make_int2((int)(unsigned)w, (int)(w >> 32));
                    }
                }
                // a lane whose grid point the region misses reads a zero, so
                // the loads carry no condition and nothing consumes one
                // before the last is issued
                T v[kFoldBatch];
#pragma unroll
                for (int u = 0; u < kFoldBatch; ++u) {
                    const int q = p + u * stride;
                    const int2 pr = prs[u];
                    const int ex = (((pr.y & 1023) + cx) & (n - 1));
                    const int ey = DA >= 2 ? ((((pr.y >> 10) & 1023) + cy) & (n - 1)) : 0;
                    const int ez = DA == 3 ? ((((pr.y >> 20) & 1023) + cz) & (n - 1)) : 0;
                    const bool in = q < p1 && ex < L && ey < L && ez < L;
                    const global_ptr<T> at = src + ((size_t)pr.x * vol + ez * L2 + ey * L + ex);
                    v[u] = *(in ? at : as_global(&kZeroValue<T>));
                }
#pragma unroll
                for (int u = 0; u < kFoldBatch; ++u) s += (double)v[u];
            }
        } else {
            for (int p = first; p < p1; p += stride) {
                const int2 pr = pair_at(p);
                const global_ptr<T> reg = src + (size_t)pr.x * vol;
                const int bx = pr.y & 1023, by = (pr.y >> 10) & 1023, bz = (pr.y >> 20) & 1023;
                const int ex0 = (bx + cx) & (n - 1);
                const int ey0 = DA >= 2 ? (by + cy) & (n - 1) : 0;
                const int ez0 = DA == 3 ? (bz + cz) & (n - 1) : 0;
                for (int ez = ez0; ez < (DA == 3 ? L : 1); ez += n)
                    for (int ey = ey0; ey < (DA >= 2 ? L : 1); ey += n)
                        for (int ex = ex0; ex < L; ex += n) s += (double)reg[ez * L2 + ey * L + ex];
            }
        }
        return s;
    };
    if (cells >= kBlock) {
        for (int c = (int)threadIdx.x; c < cells; c += kBlock)
            grid[grid_index(d, c)] = static_cast<T>(cell_sum(c, p0, 1));
        return;
    }
    const int S = kBlock / cells;  // cells is a power of two below kBlock
    const int c = (int)threadIdx.x % cells, split = (int)threadIdx.x / cells;
    part[threadIdx.x] = cell_sum(c, p0 + split, S);
    __syncthreads();
    if (split == 0) {
        double s = part[c];
        for (int k = 1; k < S; ++k) s += part[k * cells + c];
        grid[grid_index(d, c)] = static_cast<T>(s);
    }
}

// ------------------------------------------------------------------ convolve
// Forward FFT, multiplication by the real, even per-axis multiplier and
// inverse FFT of NP complex lines of length n held in LDS (src; dst is
// scratch): radix-2 Stockham.  Because the multiplier is real and even,
// filtering x + i y equals filtering x and y separately, so each complex
// line carries two real lines.  Returns the buffer that holds the result.
template <typename T, int LOGN>
__device__ __forceinline__ typename Cplx<T>::type *filter_lines(typename Cplx<T>::type *src,
                                                                typename Cplx<T>::type *dst,
                                                                int NP, const T *__restrict__ bconv,
                                                                const typename Cplx<T>::type *__restrict__ tw) {
    using C = typename Cplx<T>::type;
    constexpr int n = 1 << LOGN;
    // with n/2 dividing the workgroup size a thread keeps one butterfly
    // column j = threadIdx.x mod n/2 in every stage: its LOGN twiddles and
    // its multiplier values are loaded once, into registers
    constexpr bool kFixedColumn = (n / 2) <= kBlock;
    C twr[kFixedColumn ? LOGN : 1];
    if constexpr (kFixedColumn) {
        const int j = (int)threadIdx.x & (n / 2 - 1);
#pragma unroll
        for (int st = 0; st < LOGN; ++st) twr[st] = tw[(j & ((1 << st) - 1)) << (LOGN - 1 - st)];
    }
    // butterflies of stage st (sub-transform length Ns = 2^st); inverse:
    // conjugate twiddles
    auto stage = [&](int st, bool inverse) {
        const int Ns = 1 << st;
        for (int e = threadIdx.x; e < NP * (n / 2); e += kBlock) {
            const int ql = e >> (LOGN - 1), j = e & (n / 2 - 1);
            const int k = j & (Ns - 1);
            const C a = src[ql * n + j];
            const C b0 = src[ql * n + j + n / 2];
            C w;
            if constexpr (kFixedColumn) w = twr[st];
            else w = tw[k * (n / (2 * Ns))];
            if (inverse) w.y = -w.y;
            C b;
            b.x = b0.x * w.x - b0.y * w.y;
            b.y = b0.x * w.y + b0.y * w.x;
            const int idx = ((j - k) << 1) + k;
            dst[ql * n + idx] = C{a.x + b.x, a.y + b.y};
            dst[ql * n + idx + Ns] = C{a.x - b.x, a.y - b.y};
        }
        __syncthreads();
        C *t = src; src = dst; dst = t;
    };
    // forward transform, X_k = sum_u x_u exp(-2 pi i k u / n)
#pragma unroll
    for (int st = 0; st < LOGN; ++st) stage(st, false);
    for (int e = threadIdx.x; e < NP * n; e += kBlock) {
        const T f = bconv[e & (n - 1)];
        C v = src[e];
        v.x *= f; v.y *= f;
        src[e] = v;
    }
    __syncthreads();
    // inverse transform (no 1/n: folded into the multiplier)
#pragma unroll
    for (int st = 0; st < LOGN; ++st) stage(st, true);
    return src;
}

// ---- register-resident transforms of 64 to 256 points
// DFT of R = 8 or 16 values held in registers (radix 2, decimation in
// time, unrolled: every index is a compile-time constant).  Forward:
// A_k = sum_u a_u exp(-2 pi i u k / R); INV: the conjugate exponent.  The
// twiddles are exp(-+2 pi i j / 16), cos and sin of multiples of pi / 8.
__host__ __device__ constexpr int bit_reverse(int i, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_reg(typename Cplx<T>::type (&a)[R]) {
    using C = typename Cplx<T>::type;
    static_assert(R == 2 || R == 4 || R == 8 || R == 16, "2 to 16 points");
    constexpr int LR = R == 2 ? 1 : (R == 4 ? 2 : (R == 8 ? 3 : 4));
    constexpr double c16[8] = {1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
                               0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674};
    constexpr double s16[8] = {0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674,
                               1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977};
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int j = bit_reverse(i, LR);
        if (j > i) {
            const C t = a[i];
            a[i] = a[j];
            a[j] = t;
        }
    }
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
        for (int i = 0; i < R; i += len) {
#pragma unroll
            for (int k = 0; k < len / 2; ++k) {
                const T wr = (T)c16[k * (16 / len)];
                const T wi = INV ? (T)s16[k * (16 / len)] : -(T)s16[k * (16 / len)];
                const C u = a[i + k], v0 = a[i + k + len / 2];
                C v;
                if (k == 0) {
                    v = v0;
                } else {
                    v.x = v0.x * wr - v0.y * wi;
                    v.y = v0.x * wi + v0.y * wr;
                }
                a[i + k] = C{u.x + v.x, u.y + v.y};
                a[i + k + len / 2] = C{u.x - v.x, u.y - v.y};
            }
        }
    }
}

// exp(-2 pi i p / n) from the plan's table of the first n/2 powers (real
// and imaginary parts interleaved), read without a branch: the second half
// is the first negated
template <typename C, typename T>
__device__ __forceinline__ C twiddle_pow(global_ptr<T> tw, int p, int n) {
    p &= n - 1;
    const int i = p & (n / 2 - 1);
    const T sgn = p < n / 2 ? T(1) : T(-1);
    return C{sgn * tw[2 * i], sgn * tw[2 * i + 1]};
}

// Axis pass for n = R1 R2 = 64, 128 or 256 (R1 = 8 or 16, R2 = 8 or 16):
// forward transform, multiplier, inverse transform of NP complex lines (two
// real lines each) with one LDS exchange per direction.  Index u = u1 +
// R1 u2 and k = k2 + R2 k1: thread t of a line first transforms its u1 = t
// column over u2 (R2 points), multiplies by exp(-2 pi i u1 k2 / n) and
// writes it to LDS; thread t < R2 then transforms the k2 = t row over u1
// (R1 points), which gives X at k = t + R2 k1, applies the multiplier there,
// and runs the inverse steps in the opposite order (inverse over k1,
// conjugate twiddle, exchange, inverse over k2).  The lanes of a workgroup
// map to (line, t) with consecutive lanes on neighbouring lines for the
// strided axes (their reads are then contiguous across lanes) and on
// neighbouring t for axis 0.
template <typename T, int LOGN>
__global__ __launch_bounds__(kBlock) void convolve4_kernel(const WinInst *__restrict__ insts,
                                                           const int32_t *__restrict__ members,
                                                           const int32_t *__restrict__ prefix,
                                                           int cnt, int axis) {
    using C = typename Cplx<T>::type;
    constexpr int n = 1 << LOGN, R1 = 1 << ((LOGN + 1) / 2), R2 = 1 << (LOGN / 2);
    constexpr int NP = kBlock / R1;  // complex lines per workgroup
    // padded exchange rows (RS) and lines (LS odd: lanes on neighbouring
    // lines, as on the strided axes, then meet different LDS banks)
    constexpr int RS = R2 + 1, LS = R1 * RS + 1;
    __shared__ C xl[NP * LS];
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    T *__restrict__ grid = static_cast<T *>(wi.grid);
    const global_ptr<T> gg = as_global(static_cast<const T *>(grid));
    const global_ptr<T> bconv = as_global(static_cast<const T *>(wi.bconv));
    const global_ptr<T> tw = as_global(static_cast<const T *>(wi.twiddle));
    int nlines = 1;
    for (int d = 1; d < wi.dA; ++d) nlines *= n;
    const int ls = LOGN * axis;  // stride s = n^axis = 2^ls
    const size_t s = (size_t)1 << ls;
    const bool contiguous = axis == 0;
    // strided axes: lane groups of NP take columns t in the order 0, R1/2,
    // 1, R1/2 + 1, ..., so that every wave holds as many columns t < R2 (the
    // ones that do the middle step) as the others
    const int tq = (int)threadIdx.x / NP;
    const int q = contiguous ? (int)threadIdx.x / R1 : (int)threadIdx.x % NP;
    const int t = contiguous ? (int)threadIdx.x % R1 : (tq & 1) * (R1 / 2) + (tq >> 1);
    const int r0 = 2 * (loc.lb * NP + q), r1 = r0 + 1;
    auto base_of = [&](int r) -> size_t {
        const size_t hi = (size_t)(r >> ls), lo = (size_t)(r & (int)(s - 1));
        return hi * s * n + lo;
    };
    const size_t b0 = base_of(r0), b1 = base_of(r1);
    const bool in0 = r0 < nlines, in1 = r1 < nlines;
    C *xq = xl + q * LS;
    // forward over u2 for u1 = t, twiddle, exchange
    C a[R2];
#pragma unroll
    for (int u2 = 0; u2 < R2; ++u2) {
        const size_t off = (size_t)(t + R1 * u2) * s;
        a[u2] = C{load_or_zero(gg + (b0 + off), in0), load_or_zero(gg + (b1 + off), in1)};
    }
    dft_reg<T, R2, false>(a);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
        const C w = twiddle_pow<C>(tw, t * k2, n);
        const C v = a[k2];
        xq[t * RS + k2] = C{v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x};
    }
    __syncthreads();
    if (t < R2) {
        // forward over u1 for k2 = t: X at k = t + R2 k1; multiplier; inverse
        C b[R1];
#pragma unroll
        for (int u1 = 0; u1 < R1; ++u1) b[u1] = xq[u1 * RS + t];
        dft_reg<T, R1, false>(b);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            const T f = bconv[t + R2 * k1];
            b[k1].x *= f;
            b[k1].y *= f;
        }
        dft_reg<T, R1, true>(b);
#pragma unroll
        for (int u1 = 0; u1 < R1; ++u1) {
            const C w = twiddle_pow<C>(tw, u1 * t, n);  // conjugated below
            const C v = b[u1];
            xq[u1 * RS + t] = C{v.x * w.x + v.y * w.y, v.y * w.x - v.x * w.y};
        }
    }
    __syncthreads();
    // inverse over k2 for u1 = t: the line at u = t + R1 u2 (the multiplier
    // carries the 1/n)
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) a[k2] = xq[t * RS + k2];
    dft_reg<T, R2, true>(a);
#pragma unroll
    for (int u2 = 0; u2 < R2; ++u2) {
        const size_t off = (size_t)(t + R1 * u2) * s;
        if (in0) grid[b0 + off] = a[u2].x;
        if (in1) grid[b1 + off] = a[u2].y;
    }
}

// One pass along `axis` (element stride n^axis) of the n^d_A real grid of
// each instance, NP complex lines (2 NP real lines) per workgroup.
template <typename T, int LOGN>
__global__ __launch_bounds__(kBlock) void convolve_kernel(const WinInst *__restrict__ insts,
                                                          const int32_t *__restrict__ members,
                                                          const int32_t *__restrict__ prefix,
                                                          int cnt, int axis, int NP) {
    using C = typename Cplx<T>::type;
    constexpr int n = 1 << LOGN;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *bufA = reinterpret_cast<C *>(smem_raw);
    C *bufB = bufA + NP * n;
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    T *__restrict__ grid = static_cast<T *>(wi.grid);
    const T *__restrict__ bconv = static_cast<const T *>(wi.bconv);
    const C *__restrict__ tw = static_cast<const C *>(wi.twiddle);
    int nlines = 1;
    for (int t = 1; t < wi.dA; ++t) nlines *= n;
    const int ls = LOGN * axis;  // stride s = n^axis = 2^ls
    const int s = 1 << ls;
    const int q0 = loc.lb * NP;
    const bool contiguous = (s == 1);
    auto base_of = [&](int r) -> size_t {
        const size_t hi = (size_t)(r >> ls), lo = (size_t)(r & (s - 1));
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
    const C *res = filter_lines<T, LOGN>(bufA, bufB, NP, bconv, tw);
    for (int e = threadIdx.x; e < NP * n; e += kBlock) {
        int ql, u;
        if (contiguous) { ql = e / n; u = e % n; } else { u = e / NP; ql = e % NP; }
        const int r0 = 2 * (q0 + ql), r1 = r0 + 1;
        const C v = res[ql * n + u];
        if (r0 < nlines) grid[base_of(r0) + (size_t)u * s] = v.x;
        if (r1 < nlines) grid[base_of(r1) + (size_t)u * s] = v.y;
    }
}

// Small grids (n <= 32, d_A >= 2): a pass along one axis is the circular
// convolution with the real, even taps c_d = sum_k b_k cos(2 pi k d / n) of
// the multiplier b (its inverse transform, from the plan), n multiply-adds
// per value and no FFT stages.  The plane kernel does axes 0 and 1 of one
// n x n plane (plane z = workgroup index in 3-D, the whole grid in 2-D)
// with the plane in LDS between the passes; the axis-2 kernel takes the n
// columns of one y (workgroup index) along z.
template <typename T, int LOGN>
__global__ __launch_bounds__(kBlock) void convolve_plane_kernel(const WinInst *__restrict__ insts,
                                                                const int32_t *__restrict__ members,
                                                                const int32_t *__restrict__ prefix,
                                                                int cnt) {
    constexpr int n = 1 << LOGN, NN = n * n;
    __shared__ T a[NN], b[NN];
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    T *__restrict__ plane = static_cast<T *>(wi.grid) + (size_t)loc.lb * NN;
    const T *__restrict__ taps = static_cast<const T *>(wi.ctaps);
    const global_ptr<T> gp = as_global(plane);
    fill_lds<(NN + kBlock - 1) / kBlock, T>(NN, kBlock, [&](int e) { return gp[e]; }, [&](int e, T v) { a[e] = v; });
    // the taps are the same for every lane: scalar registers, so that a
    // tap costs one LDS read (of the line) instead of two
    T cr[n];
#pragma unroll
    for (int v = 0; v < n; ++v) cr[v] = taps[v];
    __syncthreads();
    for (int e = threadIdx.x; e < NN; e += kBlock) {  // along x: sum_v c_v a[x - v]
        const int x = e & (n - 1), row = e - x;
        T acc = T(0);
#pragma unroll
        for (int v = 0; v < n; ++v) acc += cr[v] * a[row + ((x - v) & (n - 1))];
        b[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NN; e += kBlock) {  // along y
        const int x = e & (n - 1), y = e >> LOGN;
        T acc = T(0);
#pragma unroll
        for (int v = 0; v < n; ++v) acc += cr[v] * b[((y - v) & (n - 1)) * n + x];
        plane[e] = acc;
    }
}

template <typename T, int LOGN>
__global__ __launch_bounds__(kBlock) void convolve_z_kernel(const WinInst *__restrict__ insts,
                                                            const int32_t *__restrict__ members,
                                                            const int32_t *__restrict__ prefix,
                                                            int cnt) {
    constexpr int n = 1 << LOGN, NN = n * n;
    __shared__ T a[NN];  // a[z][x]
    const Located loc = locate(insts, members, prefix, cnt);
    const WinInst &wi = *loc.w;
    T *__restrict__ col = static_cast<T *>(wi.grid) + (size_t)loc.lb * n;  // y = workgroup
    const T *__restrict__ taps = static_cast<const T *>(wi.ctaps);
    const global_ptr<T> gc = as_global(col);
    fill_lds<(NN + kBlock - 1) / kBlock, T>(
        NN, kBlock, [&](int e) { return gc[(size_t)(e >> LOGN) * NN + (e & (n - 1))]; },
        [&](int e, T v) { a[e] = v; });
    T cr[n];  // taps in scalar registers, as in the plane pass
#pragma unroll
    for (int v = 0; v < n; ++v) cr[v] = taps[v];
    __syncthreads();
    for (int e = threadIdx.x; e < NN; e += kBlock) {
        const int x = e & (n - 1), z = e >> LOGN;
        T acc = T(0);
#pragma unroll
        for (int v = 0; v < n; ++v) acc += cr[v] * a[((z - v) & (n - 1)) * n + x];
        col[(size_t)z * NN + x] = acc;
    }
}

// ------------------------------------------------------------------ combine
// out_i = beta alpha_i + sum_l eta_l tmp_l[i] in float64, windows in order
// (accumulate: out_i += the sum instead; no alpha, as for predictions at
// other points: the sum alone).  tmp_l holds window l's
// interpolated values in the caller's point order (the gather kernels write
// them there: scattered writes, which the caches merge, cost less than the
// line-sized random reads of reading them back through the inverse
// permutation).  Blocks: ceil(N / kCombineSpan) per instance.
constexpr int kConvolveDirectMax = 32;  // largest n convolved by direct taps
constexpr int kCombinePerThread = 2;
constexpr int kCombineSpan = kCombinePerThread * kBlock;

template <typename T>
__global__ __launch_bounds__(kBlock) void combine_kernel(const CombInst *__restrict__ cis,
                                                         const CombineWin *__restrict__ wins,
                                                         const int32_t *__restrict__ prefix,
                                                         int cnt) {
    constexpr int E = kCombinePerThread;
    const int q = __builtin_amdgcn_readfirstlane(find_member(prefix, cnt, blockIdx.x));
    const CombInst ci = cis[q];
    const int i0 = (blockIdx.x - prefix[q]) * kCombineSpan + threadIdx.x;
    double s[E], av[E];  // av: alpha, kept for the CG partial sum below
    {
        const global_ptr<double> ga = as_global(ci.alpha), go = as_global(ci.out);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = i0 + e * kBlock;
            av[e] = load_or_zero(ga + i, ci.alpha != nullptr && i < ci.N);
            const double o = load_or_zero(go + i, ci.accumulate && i < ci.N);
            s[e] = ci.accumulate ? o : ci.beta * av[e];
        }
    }
    // windows four at a time: their values' loads all go out before the
    // sums, which add the windows in order
    constexpr int PB = 4;
    for (int l0 = 0; l0 < ci.P; l0 += PB) {
        double eta[PB];
        T v[PB][E];
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            const bool has = l0 + u < ci.P;
            const CombineWin cw = wins[ci.win0 + min(l0 + u, ci.P - 1)];
            eta[u] = has ? cw.eta : 0.0;
            const global_ptr<T> tmp = as_global(static_cast<const T *>(cw.tmp));
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int i = i0 + e * kBlock;
                v[u][e] = load_or_zero(tmp + i, has && i < ci.N);
            }
        }
#pragma unroll
        for (int u = 0; u < PB; ++u)
            if (l0 + u < ci.P) {
#pragma unroll
                for (int e = 0; e < E; ++e) s[e] += eta[u] * (double)v[u][e];
            }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = i0 + e * kBlock;
        if (i < ci.N) ci.out[i] = s[e];
    }
    if (ci.hook.partial == nullptr) return;
    // CG: this workgroup's partial sum of p.q (p = alpha, q = out), added
    // by the step-length kernel in index order
    __shared__ double red[kBlock / 64];
    double v = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = i0 + e * kBlock;
        if (i < ci.N) v += av[e] * s[e];
    }
    v = block_sum_f64(v, red);
    if (threadIdx.x == 0) ci.hook.partial[blockIdx.x - prefix[q]] = v;
}

// ================================================================== host side
namespace {

int ilog2(int n) {
    int l = 0;
    while ((1 << (l + 1)) <= n) ++l;
    return l;
}
// n = 64 .. 256 (float64: up to 128, whose exchange fits 64 KB of LDS) go
// through the register-resident transform kernel
bool convolve_four_step(int n, int elem_bytes) {
    return (n == 64 || n == 128 || n == 256) && (elem_bytes == 4 || n <= 128);
}

template <int DA>
struct CellTileOf {
    static constexpr int value = DA == 3 ? 4 : (DA == 2 ? 16 : 64);
};
template <int DA, int W>
constexpr bool cell_supported() {
    return DA == 3 ? W <= 6 : (DA == 2 ? W <= 8 : W <= 16);
}

template <typename K>
void launch_k(K kernel, const BatchGroup &g, size_t shm, const WinInst *insts, hipStream_t s) {
    if (g.blocks <= 0) return;
    hipLaunchKernelGGL(kernel, dim3((unsigned)g.blocks), dim3(kBlock), shm, s, insts, g.members,
                       g.prefix, g.cnt);
    ANOVA_HIP_CHECK(hipGetLastError());
}

size_t region_elems(int dA, int tile, int W) {
    const size_t L = (size_t)tile + W - 1;
    size_t vol = L;
    if (dA >= 2) vol *= L;
    if (dA >= 3) vol *= L;
    return vol;
}

template <typename T, int DA, int W>
void spread_pt_launch(const BatchGroup &g, const WinInst *insts, hipStream_t s) {
    launch_k(spread_pt_kernel<T, DA, W>, g, region_elems(DA, g.tile, W) * 8, insts, s);
}
template <typename T, int DA, int W>
void gather_pt_launch(const BatchGroup &g, const WinInst *insts, hipStream_t s) {
    launch_k(gather_pt_kernel<T, DA, W>, g, region_elems(DA, g.tile, W) * sizeof(T), insts, s);
}
template <typename K>
void launch_nt(K kernel, int nt, const BatchGroup &g, const WinInst *insts, hipStream_t s) {
    if (g.blocks <= 0) return;
    hipLaunchKernelGGL(kernel, dim3((unsigned)g.blocks), dim3(nt), 0, s, insts, g.members,
                       g.prefix, g.cnt);
    ANOVA_HIP_CHECK(hipGetLastError());
}
template <int DA, int W>
void spread_cell_launch(const BatchGroup &g, const WinInst *insts, hipStream_t s) {
    if constexpr (DA == 3 && (W == 8 || W == 12)) {
        if (g.tile != kWideTile)
            throw Error{ANOVA_E_INVALID, "wide per-cell kernels take 4^3-cell tiles"};
        if constexpr (W == 12) launch_nt(spread_mfma_kernel<W>, kMfmaThreads, g, insts, s);
        else launch_nt(spread_wide_kernel<W>, kWideThreads, g, insts, s);
    } else if constexpr (cell_supported<DA, W>()) {
        constexpr int TILE = CellTileOf<DA>::value;
        constexpr int S = kBlock / CellShape<DA, TILE>::cells;
        launch_k(spread_cell_kernel<DA, W, TILE, S>, g, 0, insts, s);
    } else {
        throw Error{ANOVA_E_INVALID, "per-cell spreading does not support this window width"};
    }
}
template <int DA, int W>
void gather_cell_launch(const BatchGroup &g, const WinInst *insts, hipStream_t s) {
    if constexpr (DA == 3 && (W == 8 || W == 12)) {
        if (g.tile != kWideTile)
            throw Error{ANOVA_E_INVALID, "wide per-cell kernels take 4^3-cell tiles"};
        if constexpr (W == 12) launch_nt(gather_mfma_kernel<W>, kMfmaThreads, g, insts, s);
        else launch_nt(gather_wide_kernel<W>, kWideThreads, g, insts, s);
    } else if constexpr (cell_supported<DA, W>()) {
        constexpr int TILE = CellTileOf<DA>::value;
        constexpr int S = kBlock / CellShape<DA, TILE>::cells;
        launch_k(gather_cell_kernel<DA, W, TILE, S>, g, 0, insts, s);
    } else {
        throw Error{ANOVA_E_INVALID, "per-cell gathering does not support this window width"};
    }
}

#define ANOVA_W_SWITCH(Wv, CALL)                                                        \
    switch (Wv) {                                                                       \
        case 4: { constexpr int W_ = 4; CALL; } break;                                  \
        case 6: { constexpr int W_ = 6; CALL; } break;                                  \
        case 8: { constexpr int W_ = 8; CALL; } break;                                  \
        case 10: { constexpr int W_ = 10; CALL; } break;                                \
        case 12: { constexpr int W_ = 12; CALL; } break;                                \
        case 14: { constexpr int W_ = 14; CALL; } break;                                \
        case 16: { constexpr int W_ = 16; CALL; } break;                                \
        default: throw Error{ANOVA_E_INVALID, "window width out of range"};             \
    }
#define ANOVA_DA_SWITCH(DAv, CALL)                                                      \
    switch (DAv) {                                                                      \
        case 1: { constexpr int DA_ = 1; CALL; } break;                                 \
        case 2: { constexpr int DA_ = 2; CALL; } break;                                 \
        case 3: { constexpr int DA_ = 3; CALL; } break;                                 \
        default: throw Error{ANOVA_E_INVALID, "d_A out of range"};                      \
    }

template <int DA, int W>
int spread_cell_blocks_per_cu() {
    int nb = 0;
    if constexpr (DA == 3 && (W == 8 || W == 12)) {
        if constexpr (W == 12)
            ANOVA_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, reinterpret_cast<const void *>(spread_mfma_kernel<W>), kMfmaThreads, 0));
        else
            ANOVA_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, reinterpret_cast<const void *>(spread_wide_kernel<W>), kWideThreads, 0));
    } else if constexpr (cell_supported<DA, W>()) {
        constexpr int TILE = CellTileOf<DA>::value;
        constexpr int S = kBlock / CellShape<DA, TILE>::cells;
        ANOVA_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(spread_cell_kernel<DA, W, TILE, S>), kBlock, 0));
    }
    return nb;
}

template <typename T>
void spread_group(const BatchGroup &g, const WinInst *insts, hipStream_t s) {
    if (g.cell) {
        if constexpr (std::is_same<T, float>::value) {
            ANOVA_DA_SWITCH(g.dA, ANOVA_W_SWITCH(g.W, (spread_cell_launch<DA_, W_>(g, insts, s))));
        } else {
            if (g.dA != 3 || g.tile != 4 || (g.W != 4 && g.W != 6))
                throw Error{ANOVA_E_INVALID, "float64 per-cell kernels take d_A = 3, W <= 6"};
            if (g.W == 4) launch_k(spread_cell64_kernel<4>, g, 0, insts, s);
            else launch_k(spread_cell64_kernel<6>, g, 0, insts, s);
        }
    } else {
        ANOVA_DA_SWITCH(g.dA, ANOVA_W_SWITCH(g.W, (spread_pt_launch<T, DA_, W_>(g, insts, s))));
    }
}
template <typename T>
void gather_group(const BatchGroup &g, const WinInst *insts, hipStream_t s) {
    if (g.cell) {
        if constexpr (std::is_same<T, float>::value) {
            ANOVA_DA_SWITCH(g.dA, ANOVA_W_SWITCH(g.W, (gather_cell_launch<DA_, W_>(g, insts, s))));
        } else {
            if (g.dA != 3 || g.tile != 4 || (g.W != 4 && g.W != 6))
                throw Error{ANOVA_E_INVALID, "float64 per-cell kernels take d_A = 3, W <= 6"};
            if (g.W == 4) launch_k(gather_cell64_kernel<4>, g, 0, insts, s);
            else launch_k(gather_cell64_kernel<6>, g, 0, insts, s);
        }
    } else {
        ANOVA_DA_SWITCH(g.dA, ANOVA_W_SWITCH(g.W, (gather_pt_launch<T, DA_, W_>(g, insts, s))));
    }
}
template <typename T>
void fold_group(const BatchGroup &g, const WinInst *insts, hipStream_t s) {
    ANOVA_DA_SWITCH(g.dA, (launch_k(fold_kernel<T, DA_>, g, 0, insts, s)));
}
template <typename T>
void convolve_group(const BatchGroup &g, const WinInst *insts, hipStream_t s) {
    if (g.blocks <= 0) return;
    if (g.axis < 0) {  // direct passes: axes 0 and 1 by planes (-1), axis 2 (-2)
#define ANOVA_DIRECT(LOGN)                                                                      \
    if (g.axis == -1)                                                                           \
        hipLaunchKernelGGL((convolve_plane_kernel<T, LOGN>), dim3((unsigned)g.blocks), dim3(kBlock), \
                           0, s, insts, g.members, g.prefix, g.cnt);                            \
    else                                                                                        \
        hipLaunchKernelGGL((convolve_z_kernel<T, LOGN>), dim3((unsigned)g.blocks), dim3(kBlock),   \
                           0, s, insts, g.members, g.prefix, g.cnt)
        switch (g.n) {
            case 8: ANOVA_DIRECT(3); break;
            case 16: ANOVA_DIRECT(4); break;
            case 32: ANOVA_DIRECT(5); break;
            default: throw Error{ANOVA_E_INVALID, "direct convolution takes n <= 32"};
        }
#undef ANOVA_DIRECT
        ANOVA_HIP_CHECK(hipGetLastError());
        return;
    }
    if (convolve_four_step(g.n, (int)sizeof(T))) {
        if (g.np != kBlock / (1 << ((ilog2(g.n) + 1) / 2)))
            throw Error{ANOVA_E_INVALID, "convolution lines per workgroup do not match the kernel"};
#define ANOVA_CONV4(LOGN)                                                                     \
    hipLaunchKernelGGL((convolve4_kernel<T, LOGN>), dim3((unsigned)g.blocks), dim3(kBlock), 0, s, \
                       insts, g.members, g.prefix, g.cnt, g.axis)
        switch (g.n) {
            case 64: ANOVA_CONV4(6); break;
            case 128: ANOVA_CONV4(7); break;
            default: ANOVA_CONV4(8); break;
        }
#undef ANOVA_CONV4
        ANOVA_HIP_CHECK(hipGetLastError());
        return;
    }
    const size_t shm = 2 * (size_t)g.np * g.n * sizeof(typename Cplx<T>::type);
#define ANOVA_CONV(LOGN)                                                                  \
    hipLaunchKernelGGL((convolve_kernel<T, LOGN>), dim3((unsigned)g.blocks), dim3(kBlock), \
                       shm, s, insts, g.members, g.prefix, g.cnt, g.axis, g.np)
    switch (g.n) {
        case 8: ANOVA_CONV(3); break;
        case 16: ANOVA_CONV(4); break;
        case 32: ANOVA_CONV(5); break;
        case 64: ANOVA_CONV(6); break;
        case 128: ANOVA_CONV(7); break;
        case 256: ANOVA_CONV(8); break;
        default: throw Error{ANOVA_E_INVALID, "grid length n must be a power of two in [8, 256]"};
    }
#undef ANOVA_CONV
    ANOVA_HIP_CHECK(hipGetLastError());
}

}  // namespace

bool convolve_direct(int n, int dA) { return dA >= 2 && n <= kConvolveDirectMax; }
int convolve_lines_per_block(int n, int nq, int elem_bytes) {
    // the register-resident kernel maps its threads to (line, column)
    if (convolve_four_step(n, elem_bytes)) return kBlock / (1 << ((ilog2(n) + 1) / 2));
    // passes along y and z read, for each line position, the workgroup's
    // 2 NP neighbouring lines: 2 NP elements of 128 contiguous bytes keep
    // those reads whole cache lines (NP = 16 floats or 8 doubles); the LDS
    // holds 2 NP n complex values (32 KB at n = 128), and there are at
    // least ~64 workgroups per grid when it has that many line pairs (the
    // launches cover every window, so several grids share them)
    const int per_block = std::max(1, (elem_bytes == 4 ? 2048 : 1024) / n);
    return std::max(1, std::min(per_block, (nq + 63) / 64));
}
int cell_tile(int dA) { return dA == 3 ? 4 : (dA == 2 ? 16 : 64); }
bool cell_width_supported(int dA, int W, int precision) {
    if (precision == ANOVA_FP64) return dA == 3 && (W == 4 || W == 6);
    return dA == 3 ? (W <= 6 || W == 8 || W == 12) : (dA == 2 ? W <= 8 : W <= 16);
}
int fold_blocks(const WinInst &w) {
    int cells = w.tile;
    for (int t = 1; t < w.dA; ++t) cells *= w.tile;
    const int per = (cells >= kBlock ? 1 : kBlock / cells) * kFoldZeroPasses;
    return w.fold_act + (w.fold_len - w.fold_act + per - 1) / per;
}
int cell_resident_blocks(int dA, int W, int precision) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int>, int> cache;
    int dev = 0;
    ANOVA_HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(dev, dA, W, precision);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int nb = 0, cus = 0;
    if (precision == ANOVA_FP64) {
        const void *k = W == 4 ? reinterpret_cast<const void *>(spread_cell64_kernel<4>)
                               : reinterpret_cast<const void *>(spread_cell64_kernel<6>);
        ANOVA_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kBlock, 0));
    } else {
        ANOVA_DA_SWITCH(dA, ANOVA_W_SWITCH(W, (nb = spread_cell_blocks_per_cu<DA_, W_>())));
    }
    ANOVA_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int r = std::max(1, nb) * std::max(1, cus);
    cache[key] = r;
    return r;
}
int cell_point_splits(int dA, int W, int precision) {
    // lanes of a cell that split its points (the wide 3-D kernels and the
    // float64 ones split the support instead: every lane of a cell walks
    // all of its points)
    if (precision == ANOVA_FP64) return 1;
    if (dA == 3) return W <= 6 ? 4 : 1;
    return dA == 2 ? 1 : 4;
}
int combine_span() { return kCombineSpan; }
int permute_span() { return kPermuteSpan; }

void run_group(const BatchGroup &g, int precision, const WinInst *insts, hipStream_t s) {
    const bool f64 = precision == ANOVA_FP64;
    switch (g.stage) {
        case kStagePermute:
            if (f64) launch_k(permute_kernel<double>, g, 0, insts, s);
            else launch_k(permute_kernel<float>, g, 0, insts, s);
            break;
        case kStageSpread:
            if (f64) spread_group<double>(g, insts, s); else spread_group<float>(g, insts, s);
            break;
        case kStageTileSum:
            if (f64) launch_k(tile_sum_kernel<double>, g, 0, insts, s);
            else launch_k(tile_sum_kernel<float>, g, 0, insts, s);
            break;
        case kStageFold:
            if (f64) fold_group<double>(g, insts, s); else fold_group<float>(g, insts, s);
            break;
        case kStageConvolve:
            if (f64) convolve_group<double>(g, insts, s); else convolve_group<float>(g, insts, s);
            break;
        case kStageGather:
            if (f64) gather_group<double>(g, insts, s); else gather_group<float>(g, insts, s);
            break;
        default: throw Error{ANOVA_E_INVALID, "unknown stage"};
    }
}

void run_combine(const CombInst *cis, const CombineWin *wins, const int32_t *prefix, int cnt,
                 int blocks, int precision, hipStream_t s) {
    if (blocks <= 0) return;
    if (precision == ANOVA_FP64)
        hipLaunchKernelGGL(combine_kernel<double>, dim3((unsigned)blocks), dim3(kBlock), 0, s, cis,
                           wins, prefix, cnt);
    else
        hipLaunchKernelGGL(combine_kernel<float>, dim3((unsigned)blocks), dim3(kBlock), 0, s, cis,
                           wins, prefix, cnt);
    ANOVA_HIP_CHECK(hipGetLastError());
}

}  // namespace anova
