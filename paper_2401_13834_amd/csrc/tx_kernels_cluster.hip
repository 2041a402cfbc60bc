// DBSCAN over the thresholded DM-time plane (Sec. 2.5), for gfx950.
//
// The paper clusters the points (DM, time, best width, S/N) of the plane to
// remove duplicate detections of one pulse: DM is converted to dispersion
// delay (Eq. 1) so both axes are times; a point is a core point when more
// than k other points lie within radius r; clusters are the sets of points
// density-reachable from core points.  The paper finds neighbours with a
// kd-tree on the CPU; here the points are sorted by (DM index, time) and a
// point's neighbours are found by binary search in the rows of the DM indices
// whose delay lies within r (a contiguous index range, delay being monotone in
// DM), then the core points are joined with a lock-free union-find.
//
// Readings (where the paper leaves a choice): the delay is across the band
// (lowest to highest channel frequency), in samples, unrounded; neighbours
// are points other than p at Euclidean distance <= r; core: more than k
// neighbours; a non-core point within r of core points joins the cluster of
// the nearest one (ties: the first in (DM, time) order), else it is noise;
// clusters are numbered in the order of their first core point; a cluster's
// representative is its highest-S/N point (ties: the first).
#include <hipcub/hipcub.hpp>

#include "tx_internal.h"

namespace tx {

namespace {

struct Pt {
    int32_t d;
    int32_t w;
    int64_t t;
    double snr;
};
static_assert(sizeof(Pt) == sizeof(tx_cand), "point record is a tx_cand");

__global__ void keys_kernel(const Pt* __restrict__ in, int64_t n, uint64_t* __restrict__ keys,
                            int32_t* __restrict__ idx) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = (static_cast<uint64_t>(static_cast<uint32_t>(in[i].d)) << 32) | static_cast<uint32_t>(in[i].t);
    idx[i] = static_cast<int32_t>(i);
}

__global__ void gather_kernel(const Pt* __restrict__ in, const int32_t* __restrict__ perm, int64_t n,
                              Pt* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[perm[i]];
}

// seg[d] = first sorted point with DM index >= d, for d in [0, ndm].
__global__ void segments_kernel(const Pt* __restrict__ p, int64_t n, int32_t ndm, int32_t* __restrict__ seg) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d > ndm) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (p[mid].d < d) lo = mid + 1; else hi = mid;
    }
    seg[d] = static_cast<int32_t>(lo);
}

// First index in [lo, hi) whose time is >= t (times sorted within a row).
__device__ __forceinline__ int32_t lower_t(const Pt* __restrict__ p, int32_t lo, int32_t hi, int64_t t) {
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (p[mid].t < t) lo = mid + 1; else hi = mid;
    }
    return lo;
}

struct Geo {
    int32_t ndm;
    const Pt* p;
    const int32_t* seg;
    const double* x;        // delay of each DM index, samples
    const int32_t* dlo;     // DM index range within r of each DM index
    const int32_t* dhi;
    double r, r2;
    int64_t rt;             // floor(r): time offsets that can be within r
};

// Visit every neighbour q != i of point i (distance <= r): f(q, d2).
template <class F>
__device__ __forceinline__ void for_neighbours(const Geo& g, int32_t i, F f) {
    const Pt pi = g.p[i];
    if (pi.d < 0 || pi.d >= g.ndm) return;   // not a trial of the plan: no neighbours
    const double xi = g.x[pi.d];
    for (int32_t dq = g.dlo[pi.d]; dq <= g.dhi[pi.d]; ++dq) {
        const int32_t a = g.seg[dq], b = g.seg[dq + 1];
        if (a == b) continue;
        const double dx = g.x[dq] - xi;
        for (int32_t q = lower_t(g.p, a, b, pi.t - g.rt); q < b; ++q) {
            const int64_t tq = g.p[q].t;
            if (tq > pi.t + g.rt) break;
            if (q == i) continue;
            const double dt = static_cast<double>(tq - pi.t);
            const double d2 = dx * dx + dt * dt;
            if (d2 <= g.r2) f(q, d2);
        }
    }
}

__global__ void core_kernel(Geo g, int32_t n, int32_t kmin, uint8_t* __restrict__ core, int32_t* __restrict__ parent) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t cnt = 0;
    for_neighbours(g, i, [&](int32_t, double) { ++cnt; });
    core[i] = cnt > kmin ? 1 : 0;
    parent[i] = i;
}

__device__ __forceinline__ int32_t find_root(int32_t* parent, int32_t x) {
    int32_t p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
    while (p != x) {
        const int32_t gp = __atomic_load_n(&parent[p], __ATOMIC_RELAXED);
        if (gp != p) atomicCAS(&parent[x], p, gp);   // path halving; losing the race is harmless
        x = p;
        p = gp;
    }
    return x;
}

// Hook the larger root under the smaller, so every component's root ends as
// its smallest point index.
__device__ __forceinline__ void unite(int32_t* parent, int32_t a, int32_t b) {
    while (true) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b) return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(&parent[a], a, b) == a) return;
    }
}

__global__ void union_kernel(Geo g, int32_t n, const uint8_t* __restrict__ core, int32_t* parent) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !core[i]) return;
    for_neighbours(g, i, [&](int32_t q, double) {
        if (q < i && core[q]) unite(parent, i, q);
    });
}

__global__ void root_kernel(int32_t n, const uint8_t* __restrict__ core, int32_t* parent, int32_t* __restrict__ root) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    root[i] = core[i] ? find_root(parent, i) : -1;
}

// Non-core points: the root of the nearest core neighbour, or -1.
__global__ void border_kernel(Geo g, int32_t n, const uint8_t* __restrict__ core, const int32_t* __restrict__ root_in,
                              int32_t* __restrict__ root_out, int32_t* __restrict__ is_root) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (core[i]) {
        root_out[i] = root_in[i];
        is_root[i] = root_in[i] == i ? 1 : 0;
        return;
    }
    double best = 0.0;
    int32_t bq = -1;
    for_neighbours(g, i, [&](int32_t q, double d2) {
        if (core[q] && (bq < 0 || d2 < best || (d2 == best && q < bq))) {
            best = d2;
            bq = q;
        }
    });
    root_out[i] = bq < 0 ? -1 : root_in[bq];
    is_root[i] = 0;
}

// Order-preserving unsigned image of a double.
__device__ __forceinline__ unsigned long long ordered(double v) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
    return (b >> 63) ? ~b : (b | (1ull << 63));
}

__global__ void label_kernel(int32_t n, const Pt* __restrict__ p, const int32_t* __restrict__ root,
                             const int32_t* __restrict__ cid, int32_t* __restrict__ label,
                             unsigned long long* __restrict__ best) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = root[i];
    const int32_t c = r < 0 ? -1 : cid[r];
    label[i] = c;
    if (c >= 0) atomicMax(&best[c], ordered(p[i].snr));
}

__global__ void rep_kernel(int32_t n, const Pt* __restrict__ p, const int32_t* __restrict__ label,
                           const unsigned long long* __restrict__ best, int64_t* __restrict__ rep) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = label[i];
    if (c >= 0 && ordered(p[i].snr) == best[c]) atomicMin(reinterpret_cast<unsigned long long*>(&rep[c]),
                                                          static_cast<unsigned long long>(i));
}

__global__ void fill_kernel(int64_t n, unsigned long long* __restrict__ a, unsigned long long v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void count_kernel(int32_t n, const int32_t* __restrict__ cid, const int32_t* __restrict__ is_root,
                             int64_t* __restrict__ nclusters) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *nclusters = n > 0 ? cid[n - 1] + is_root[n - 1] : 0;
}

inline unsigned blocks(int64_t n, int b) { return static_cast<unsigned>((n + b - 1) / b); }

}  // namespace

// Scratch layout, each part 256-byte aligned.
struct ClusterScratch {
    size_t keys, keys2, idx, idx2, seg, core, parent, root, root2, is_root, cid, best, sort_tmp, scan_tmp, total;
};

static size_t up256(size_t v) { return (v + 255) / 256 * 256; }

static ClusterScratch cluster_layout(int64_t n, int32_t ndm) {
    ClusterScratch s{};
    size_t sort_tmp = 0, scan_tmp = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sort_tmp, static_cast<uint64_t*>(nullptr),
                                             static_cast<uint64_t*>(nullptr), static_cast<int32_t*>(nullptr),
                                             static_cast<int32_t*>(nullptr), static_cast<int>(n));
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan_tmp, static_cast<int32_t*>(nullptr),
                                           static_cast<int32_t*>(nullptr), static_cast<int>(n));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += up256(bytes);
        return at;
    };
    s.keys = take(8 * n);
    s.keys2 = take(8 * n);
    s.idx = take(4 * n);
    s.idx2 = take(4 * n);
    s.seg = take(4 * (static_cast<size_t>(ndm) + 1));
    s.core = take(n);
    s.parent = take(4 * n);
    s.root = take(4 * n);
    s.root2 = take(4 * n);
    s.is_root = take(4 * n);
    s.cid = take(4 * n);
    s.best = take(8 * n);
    s.sort_tmp = take(sort_tmp);
    s.scan_tmp = take(scan_tmp);
    s.total = o;
    return s;
}

hipError_t launch_cluster(const tx_cand* d_in, int64_t n, int32_t ndm, const double* d_x, const int32_t* d_dlo,
                          const int32_t* d_dhi, double r, int32_t kmin, tx_cand* d_sorted, int32_t* d_label,
                          int64_t* d_rep, int64_t* d_nclusters, hipStream_t st) {
    if (n == 0) {
        hipLaunchKernelGGL(count_kernel, dim3(1), dim3(64), 0, st, 0, static_cast<const int32_t*>(nullptr),
                           static_cast<const int32_t*>(nullptr), d_nclusters);
        return hipGetLastError();
    }
    const ClusterScratch L = cluster_layout(n, ndm);
    void* ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, L.total, st);
    if (e != hipSuccess) return e;
    uint8_t* w = static_cast<uint8_t*>(ws);
    auto at = [&](size_t off) { return static_cast<void*>(w + off); };
    uint64_t* keys = static_cast<uint64_t*>(at(L.keys));
    uint64_t* keys2 = static_cast<uint64_t*>(at(L.keys2));
    int32_t* idx = static_cast<int32_t*>(at(L.idx));
    int32_t* perm = static_cast<int32_t*>(at(L.idx2));
    int32_t* seg = static_cast<int32_t*>(at(L.seg));
    uint8_t* core = static_cast<uint8_t*>(at(L.core));
    int32_t* parent = static_cast<int32_t*>(at(L.parent));
    int32_t* root = static_cast<int32_t*>(at(L.root));
    int32_t* root2 = static_cast<int32_t*>(at(L.root2));
    int32_t* is_root = static_cast<int32_t*>(at(L.is_root));
    int32_t* cid = static_cast<int32_t*>(at(L.cid));
    unsigned long long* best = static_cast<unsigned long long*>(at(L.best));
    const int B = 256;
    const int32_t n32 = static_cast<int32_t>(n);
    const Pt* in = reinterpret_cast<const Pt*>(d_in);
    Pt* p = reinterpret_cast<Pt*>(d_sorted);

    hipLaunchKernelGGL(keys_kernel, dim3(blocks(n, B)), dim3(B), 0, st, in, n, keys, idx);
    size_t sort_tmp = L.scan_tmp - L.sort_tmp;
    e = hipcub::DeviceRadixSort::SortPairs(at(L.sort_tmp), sort_tmp, keys, keys2, idx, perm, n32, 0, 64, st);
    // (the sorted keys themselves are not needed: the points are gathered by index)
    if (e == hipSuccess) {
        hipLaunchKernelGGL(gather_kernel, dim3(blocks(n, B)), dim3(B), 0, st, in, perm, n, p);
        hipLaunchKernelGGL(segments_kernel, dim3(blocks(ndm + 1, B)), dim3(B), 0, st, p, n, ndm, seg);
        Geo g{ndm, p, seg, d_x, d_dlo, d_dhi, r, r * r, static_cast<int64_t>(r)};
        hipLaunchKernelGGL(core_kernel, dim3(blocks(n, B)), dim3(B), 0, st, g, n32, kmin, core, parent);
        hipLaunchKernelGGL(union_kernel, dim3(blocks(n, B)), dim3(B), 0, st, g, n32, core, parent);
        hipLaunchKernelGGL(root_kernel, dim3(blocks(n, B)), dim3(B), 0, st, n32, core, parent, root);
        hipLaunchKernelGGL(border_kernel, dim3(blocks(n, B)), dim3(B), 0, st, g, n32, core, root, root2, is_root);
        size_t scan_tmp = L.total - L.scan_tmp;
        e = hipcub::DeviceScan::ExclusiveSum(at(L.scan_tmp), scan_tmp, is_root, cid, n32, st);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fill_kernel, dim3(blocks(n, B)), dim3(B), 0, st, n, best, 0ull);
        hipLaunchKernelGGL(fill_kernel, dim3(blocks(n, B)), dim3(B), 0, st, n,
                           reinterpret_cast<unsigned long long*>(d_rep), ~0ull);
        hipLaunchKernelGGL(label_kernel, dim3(blocks(n, B)), dim3(B), 0, st, n32, p, root2, cid, d_label, best);
        hipLaunchKernelGGL(rep_kernel, dim3(blocks(n, B)), dim3(B), 0, st, n32, p, d_label, best, d_rep);
        hipLaunchKernelGGL(count_kernel, dim3(1), dim3(64), 0, st, n32, cid, is_root, d_nclusters);
        e = hipGetLastError();
    }
    const hipError_t f = hipFreeAsync(ws, st);
    return e != hipSuccess ? e : f;
}

}  // namespace tx
