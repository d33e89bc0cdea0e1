// Binning and sorting of the points on the device (the plan's first step,
// Sec. 4.2: scaled nodes x~ = (x - c) / h on the torus, each assigned to the
// cell of the oversampled grid that holds it and sorted by grid tile).
//
// The device path computes exactly what the host path computes:
//   * per point and window dimension, t = (x - c) n / h + n/2 reduced mod n,
//     its cell floor(t) and fractional offset t - floor(t), in float64 with
//     the same operations in the same order (no contraction into fused
//     multiply-adds), so both paths give the same cells and offsets;
//   * the points of each sort key (tile, or tile and cell) in increasing
//     original index: a bitonic sort of the composite keys (key << 32 | i),
//     which are distinct, so any correct sort gives the one stable order.
// The points' count per grid cell goes back to the host, which derives the
// tile and cell bookkeeping from it as it does from host points.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "anova_internal.h"

namespace anova {
namespace {

constexpr int kBinBlock = 256;
constexpr int kSortBlock = 512;           // threads of the in-LDS sorting kernels
constexpr int kSortTile = 2 * kSortBlock;  // keys sorted or merged in LDS per workgroup

// ------------------------------------------------------------------ bounds
// Per column of X (d columns): minimum and maximum as order-preserving
// integer keys, and whether any entry is not finite.
__device__ __forceinline__ unsigned long long order_key(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ __launch_bounds__(kBinBlock) void bounds_kernel(const double *__restrict__ X,
                                                            int64_t N, int64_t ld, int d,
                                                            unsigned long long *__restrict__ lo,
                                                            unsigned long long *__restrict__ hi,
                                                            int *__restrict__ bad) {
    // one column per blockIdx.y; rows strided over the x blocks
    const int t = blockIdx.y;
    unsigned long long mn = ~0ull, mx = 0ull;
    int nonfinite = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBinBlock + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * kBinBlock) {
        const double v = X[i * ld + t];
        if (!isfinite(v)) {
            nonfinite = 1;
            continue;
        }
        const unsigned long long k = order_key(v);
        mn = k < mn ? k : mn;
        mx = k > mx ? k : mx;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long a = __shfl_xor(mn, off, 64), b = __shfl_xor(mx, off, 64);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
        nonfinite |= __shfl_xor(nonfinite, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(lo + t, mn);
        atomicMax(hi + t, mx);
        if (nonfinite) atomicOr(bad, 1);
    }
}

__global__ void bounds_init_kernel(unsigned long long *lo, unsigned long long *hi, int *bad, int d) {
    const int t = threadIdx.x;
    if (t < d) {
        lo[t] = ~0ull;
        hi[t] = 0ull;
    }
    if (t == 0) *bad = 0;
}

double from_order_key(unsigned long long k) {
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    double v;
    std::memcpy(&v, &b, sizeof v);
    return v;
}

// ------------------------------------------------------------------ binning
struct BinArgs {
    int64_t N, ld;
    int dA, n;
    int feat[3];
    double center[3];
    double scale;  // n / h
};

// t = (x - c) * scale + n/2 reduced to [0, n): written without fused
// multiply-adds, as the host evaluates it
template <typename T>
__global__ __launch_bounds__(kBinBlock) void bin_kernel(const double *__restrict__ X, BinArgs a,
                                                         uint32_t *__restrict__ cellw,
                                                         T *__restrict__ frac,
                                                         int32_t *__restrict__ hist) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * kBinBlock + threadIdx.x;
    if (i >= a.N) return;
    const double nd = (double)a.n;
    uint32_t packed = 0;
    int64_t lin = 0, mul = 1;
    for (int t = 0; t < a.dA; ++t) {
        double tt = (X[i * a.ld + a.feat[t]] - a.center[t]) * a.scale + 0.5 * nd;
        tt -= nd * floor(tt / nd);
        const double cf = floor(tt);
        int cell = (int)cf;
        const double f = tt - cf;
        if (cell >= a.n) cell -= a.n;
        if (cell < 0) cell += a.n;
        frac[i * 3 + t] = static_cast<T>(f);
        packed |= (uint32_t)cell << (10 * t);
        lin += (int64_t)cell * mul;
        mul *= a.n;
    }
    for (int t = a.dA; t < 3; ++t) frac[i * 3 + t] = T(0);
    cellw[i] = packed;
    atomicAdd(hist + lin, 1);
}

// ------------------------------------------------------------------ sort
struct KeyArgs {
    int64_t N, Npad;
    int dA, tile, tpd;
    int64_t cells_per_tile;
    int dense;
};

__global__ __launch_bounds__(kBinBlock) void key_kernel(const uint32_t *__restrict__ cellw,
                                                         KeyArgs a,
                                                         unsigned long long *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * kBinBlock + threadIdx.x;
    if (i >= a.Npad) return;
    if (i >= a.N) {
        keys[i] = ~0ull;  // padding sorts last
        return;
    }
    const uint32_t w = cellw[i];
    int64_t tk = 0, lk = 0, mul = 1, lmul = 1;
    for (int t = 0; t < a.dA; ++t) {
        const int cell = (int)((w >> (10 * t)) & 1023u);
        tk += (int64_t)(cell / a.tile) * mul;
        lk += (int64_t)(cell % a.tile) * lmul;
        mul *= a.tpd;
        lmul *= a.tile;
    }
    const int64_t key = a.dense ? tk * a.cells_per_tile + lk : tk * a.cells_per_tile;
    keys[i] = ((unsigned long long)key << 32) | (unsigned long long)i;
}

// Compare-exchange of elements i and i ^ j of a bitonic merge with block
// size k (ascending where i & k == 0).
__device__ __forceinline__ void cmp_swap(unsigned long long &a, unsigned long long &b, bool up) {
    if ((a > b) == up) {
        const unsigned long long t = a;
        a = b;
        b = t;
    }
}

// Sorts (first == 1) or finishes the merge stages j < kSortTile of block
// size k (first == 0) of each workgroup's kSortTile keys in LDS.
__global__ __launch_bounds__(kSortBlock) void bitonic_lds_kernel(unsigned long long *__restrict__ keys,
                                                                  int64_t k, int first) {
    __shared__ unsigned long long s[kSortTile];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    s[threadIdx.x] = keys[base + threadIdx.x];
    s[threadIdx.x + kSortBlock] = keys[base + threadIdx.x + kSortBlock];
    __syncthreads();
    auto stage = [&](int64_t kk, int j) {
        // thread t handles the pair (lo, lo + j) with lo having bit j clear
        const int t = threadIdx.x;
        const int lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const bool up = ((base + lo) & kk) == 0;
        cmp_swap(s[lo], s[lo + j], up);
        __syncthreads();
    };
    if (first) {
        for (int kk = 2; kk <= kSortTile; kk <<= 1)
            for (int j = kk >> 1; j > 0; j >>= 1) stage(kk, j);
    } else {
        for (int j = kSortTile >> 1; j > 0; j >>= 1) stage(k, j);
    }
    keys[base + threadIdx.x] = s[threadIdx.x];
    keys[base + threadIdx.x + kSortBlock] = s[threadIdx.x + kSortBlock];
}

// One merge stage j >= kSortTile of block size k over global memory: one
// thread per pair.
__global__ __launch_bounds__(kBinBlock) void bitonic_global_kernel(unsigned long long *__restrict__ keys,
                                                                    int64_t npairs, int64_t k,
                                                                    int64_t j) {
    const int64_t t = (int64_t)blockIdx.x * kBinBlock + threadIdx.x;
    if (t >= npairs) return;
    const int64_t lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));
    const bool up = (lo & k) == 0;
    unsigned long long a = keys[lo], b = keys[lo + j];
    if ((a > b) == up) {
        keys[lo] = b;
        keys[lo + j] = a;
    }
}

// Sorted position j: the point's record (offsets and packed cells) and its
// original index.
template <typename T, typename Node>
__global__ __launch_bounds__(kBinBlock) void nodes_kernel(const unsigned long long *__restrict__ keys,
                                                           int64_t N,
                                                           const uint32_t *__restrict__ cellw,
                                                           const T *__restrict__ frac,
                                                           Node *__restrict__ nodes,
                                                           int32_t *__restrict__ perm) {
    const int64_t j = (int64_t)blockIdx.x * kBinBlock + threadIdx.x;
    if (j >= N) return;
    const int32_t i = (int32_t)(keys[j] & 0xffffffffull);
    Node nd{};
    for (int t = 0; t < 3; ++t) nd.f[t] = frac[(int64_t)i * 3 + t];
    nd.cell = cellw[i];
    nodes[j] = nd;
    perm[j] = i;
}

unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

void device_bounds(const double *X, int64_t N, int64_t ld, int d, double *lo, double *hi,
                   bool &finite, hipStream_t s) {
    DevBuf buf;
    buf.alloc(2 * sizeof(unsigned long long) * (size_t)d + sizeof(int));
    unsigned long long *dlo = buf.as<unsigned long long>(), *dhi = dlo + d;
    int *bad = reinterpret_cast<int *>(dhi + d);
    hipLaunchKernelGGL(bounds_init_kernel, dim3(1), dim3(64 * ((d + 63) / 64)), 0, s, dlo, dhi,
                       bad, d);
    const unsigned gx = std::max(1u, std::min(grid_for(N, kBinBlock), 1024u));
    hipLaunchKernelGGL(bounds_kernel, dim3(gx, (unsigned)d), dim3(kBinBlock), 0, s, X, N, ld, d,
                       dlo, dhi, bad);
    ANOVA_HIP_CHECK(hipGetLastError());
    std::vector<unsigned long long> h(2 * (size_t)d);
    int hbad = 0;
    ANOVA_HIP_CHECK(hipMemcpyAsync(h.data(), dlo, h.size() * sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, s));
    ANOVA_HIP_CHECK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    ANOVA_HIP_CHECK(hipStreamSynchronize(s));
    finite = hbad == 0;
    for (int t = 0; t < d; ++t) {
        lo[t] = from_order_key(h[t]);
        hi[t] = from_order_key(h[(size_t)d + t]);
    }
}

template <typename T>
void device_bin(const double *X, int64_t N, int64_t ld, const WindowPlan &w, DeviceBins &b,
                std::vector<int32_t> &hist, hipStream_t s) {
    size_t ncells = 1;
    for (int t = 0; t < w.dA; ++t) ncells *= (size_t)w.n;
    b.cellw.alloc((size_t)N * sizeof(uint32_t));
    b.frac.alloc((size_t)N * 3 * sizeof(T));
    b.hist.alloc(ncells * sizeof(int32_t));
    ANOVA_HIP_CHECK(hipMemsetAsync(b.hist.ptr, 0, ncells * sizeof(int32_t), s));
    BinArgs a{};
    a.N = N;
    a.ld = ld;
    a.dA = w.dA;
    a.n = w.n;
    for (int t = 0; t < 3; ++t) {
        a.feat[t] = w.feat[t];
        a.center[t] = w.center[t];
    }
    a.scale = (double)w.n / w.h;
    hipLaunchKernelGGL(bin_kernel<T>, dim3(grid_for(N, kBinBlock)), dim3(kBinBlock), 0, s, X, a,
                       b.cellw.as<uint32_t>(), b.frac.as<T>(), b.hist.as<int32_t>());
    ANOVA_HIP_CHECK(hipGetLastError());
    hist.resize(ncells);
    ANOVA_HIP_CHECK(hipMemcpyAsync(hist.data(), b.hist.ptr, ncells * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s));
    ANOVA_HIP_CHECK(hipStreamSynchronize(s));
}

template <typename T, typename Node>
void device_sort_nodes(const WindowPlan &w, int64_t N, int64_t cells_per_tile, bool dense,
                       DeviceBins &b, hipStream_t s) {
    int64_t Npad = kSortTile;
    while (Npad < N) Npad <<= 1;
    DevBuf keys;
    keys.alloc((size_t)Npad * sizeof(unsigned long long));
    unsigned long long *k = keys.as<unsigned long long>();
    KeyArgs a{};
    a.N = N;
    a.Npad = Npad;
    a.dA = w.dA;
    a.tile = w.tile;
    a.tpd = w.tiles_per_dim;
    a.cells_per_tile = cells_per_tile;
    a.dense = dense ? 1 : 0;
    hipLaunchKernelGGL(key_kernel, dim3(grid_for(Npad, kBinBlock)), dim3(kBinBlock), 0, s,
                       b.cellw.as<uint32_t>(), a, k);
    const unsigned tiles = (unsigned)(Npad / kSortTile);
    hipLaunchKernelGGL(bitonic_lds_kernel, dim3(tiles), dim3(kSortBlock), 0, s, k, (int64_t)0, 1);
    for (int64_t kk = 2 * kSortTile; kk <= Npad; kk <<= 1) {
        for (int64_t j = kk >> 1; j >= kSortTile; j >>= 1)
            hipLaunchKernelGGL(bitonic_global_kernel, dim3(grid_for(Npad / 2, kBinBlock)),
                               dim3(kBinBlock), 0, s, k, Npad / 2, kk, j);
        hipLaunchKernelGGL(bitonic_lds_kernel, dim3(tiles), dim3(kSortBlock), 0, s, k, kk, 0);
    }
    ANOVA_HIP_CHECK(hipGetLastError());
    // sized as the host path's uploads size them (whole multiples of 256
    // bytes), so both plans report the same footprint
    auto rounded = [](size_t b) { return (b + 255) & ~(size_t)255; };
    DevBuf nodes, perm;
    nodes.alloc(rounded((size_t)N * sizeof(Node)));
    perm.alloc(rounded((size_t)N * sizeof(int32_t)));
    hipLaunchKernelGGL((nodes_kernel<T, Node>), dim3(grid_for(N, kBinBlock)), dim3(kBinBlock), 0,
                       s, k, N, b.cellw.as<uint32_t>(), b.frac.as<T>(), nodes.as<Node>(),
                       perm.as<int32_t>());
    ANOVA_HIP_CHECK(hipGetLastError());
    ANOVA_HIP_CHECK(hipStreamSynchronize(s));
    b.nodes = std::move(nodes);
    b.perm = std::move(perm);
}

template void device_bin<float>(const double *, int64_t, int64_t, const WindowPlan &,
                                DeviceBins &, std::vector<int32_t> &, hipStream_t);
template void device_bin<double>(const double *, int64_t, int64_t, const WindowPlan &,
                                 DeviceBins &, std::vector<int32_t> &, hipStream_t);
template void device_sort_nodes<float, NodeF32>(const WindowPlan &, int64_t, int64_t, bool,
                                                DeviceBins &, hipStream_t);
template void device_sort_nodes<double, NodeF64>(const WindowPlan &, int64_t, int64_t, bool,
                                                 DeviceBins &, hipStream_t);

}  // namespace anova
