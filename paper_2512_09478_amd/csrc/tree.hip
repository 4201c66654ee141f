// Octree and interaction lists on the GPU (Section 2.2, first step: an
// octree whose leaves hold at most M points; the near and far zones that the
// passes use).  All integer work is exact and deterministic:
//
//   root cube -> FP64 quantisation to 21-bit cells -> 63-bit Morton keys ->
//   stable LSD radix sort of (key, index) -> level-by-level split of the
//   sorted key runs -> colleagues by binary search on per-level box keys ->
//   V list as a dense table per octant-local offset slot, coarse adjacent
//   leaves top-down, X lists, and U/W by transposition; every CSR row is
//   sorted ascending.
#include <algorithm>

#include "common.h"

namespace kifmm {

namespace {

constexpr int TB = 256;
constexpr int64_t kSmallTreeN = 131072;   // trees of at most this many points: levels in one block
inline int nblocks(int64_t n, int per = TB) { return int((n + per - 1) / per); }

struct LevelTable {
    int start[kMaxLevels + 1];
    int count[kMaxLevels + 1];
};

__device__ inline uint64_t spread21(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ inline uint64_t morton3(uint64_t x, uint64_t y, uint64_t z) {
    return (spread21(x) << 2) | (spread21(y) << 1) | spread21(z);
}

__device__ inline uint64_t lane_lt_mask() {
    unsigned l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// ----------------------------------------------------------------- bbox
__global__ void k_bbox(const double* __restrict__ x, int64_t N, double* __restrict__ part,
                       int* __restrict__ bad) {
    __shared__ double s[6][TB];
    double mn[3] = {1e308, 1e308, 1e308}, mx[3] = {-1e308, -1e308, -1e308};
    int nb = 0;
    for (int64_t i = blockIdx.x * int64_t(TB) + threadIdx.x; i < N; i += int64_t(gridDim.x) * TB) {
        for (int d = 0; d < 3; ++d) {
            double v = x[3 * i + d];
            if (!isfinite(v)) nb = 1;
            mn[d] = fmin(mn[d], v);
            mx[d] = fmax(mx[d], v);
        }
    }
    if (nb) atomicOr(bad, 1);
    for (int d = 0; d < 3; ++d) {
        s[d][threadIdx.x] = mn[d];
        s[3 + d][threadIdx.x] = mx[d];
    }
    __syncthreads();
    for (int w = TB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int d = 0; d < 3; ++d) {
                s[d][threadIdx.x] = fmin(s[d][threadIdx.x], s[d][threadIdx.x + w]);
                s[3 + d][threadIdx.x] = fmax(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// ----------------------------------------------------------------- keys
// k_d = clamp(floor((x_d - lo_d) * 2^21 / s), 0, 2^21 - 1): one rounded FP64
// subtraction and an exact power-of-two scaling, as on the host side of any
// checker, so the keys are bit-reproducible.
__global__ void k_keys(const double* __restrict__ x, int64_t N, double lo0, double lo1, double lo2,
                       double scale, double side, int check_root, uint64_t* __restrict__ keys,
                       uint32_t* __restrict__ idx, int* __restrict__ bad) {
    int64_t i = blockIdx.x * int64_t(TB) + threadIdx.x;
    if (i >= N) return;
    const double lo[3] = {lo0, lo1, lo2};
    uint64_t k[3];
    int b = 0;
    for (int d = 0; d < 3; ++d) {
        double v = x[3 * i + d];
        if (!isfinite(v)) b = 1;
        if (check_root && (v < lo[d] || v > lo[d] + side)) b = 1;
        double f = floor(__dmul_rn(__dsub_rn(v, lo[d]), scale));
        f = fmin(fmax(f, 0.0), double((1 << kBits) - 1));
        k[d] = b ? 0 : uint64_t(f);
    }
    if (b) atomicOr(bad, 1);
    keys[i] = morton3(k[0], k[1], k[2]);
    idx[i] = uint32_t(i);
}

// ----------------------------------------------------------------- re-sort from the previous order
// Points that move between builds keep most of their order.  The order is by
// (key, caller index), a total order, so the sorted result does not depend on
// how it is reached: the keys are formed in the previous sorted order, the
// points out of order with a near neighbour in that sequence (D) are taken
// out, the rest (R) is checked to be sorted, D is sorted, and the two are
// merged.

// (key, index) strictly before (key2, index2)
__device__ inline bool kv_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

__global__ void k_keys_prev(const double* __restrict__ x, int64_t N, double lo0, double lo1, double lo2,
                            double scale, double side, int check_root, const int* __restrict__ prev,
                            uint64_t* __restrict__ keys, uint32_t* __restrict__ idx, int* __restrict__ bad) {
    int64_t i = blockIdx.x * int64_t(TB) + threadIdx.x;
    if (i >= N) return;
    const int64_t j = prev[i];
    const double lo[3] = {lo0, lo1, lo2};
    uint64_t k[3];
    int b = 0;
    for (int d = 0; d < 3; ++d) {
        double v = x[3 * j + d];
        if (!isfinite(v)) b = 1;
        if (check_root && (v < lo[d] || v > lo[d] + side)) b = 1;
        double f = floor(__dmul_rn(__dsub_rn(v, lo[d]), scale));
        f = fmin(fmax(f, 0.0), double((1 << kBits) - 1));
        k[d] = b ? 0 : uint64_t(f);
    }
    if (b) atomicOr(bad, 1);
    keys[i] = morton3(k[0], k[1], k[2]);
    idx[i] = uint32_t(j);
}

// flag[i] = 1 when element i is out of order with any element at most
// kResortWindow places away (so that a group of up to that many points that
// moved together past others is taken out whole); flag[N] = 0, and the error
// word of the later order check starts at 0
constexpr int kResortWindow = 8;
__global__ void k_displaced(const uint64_t* __restrict__ k, const uint32_t* __restrict__ v, int64_t N,
                            int* __restrict__ flag, int* __restrict__ err) {
    int64_t i = blockIdx.x * int64_t(TB) + threadIdx.x;
    if (i > N) return;
    if (i == N) {
        flag[N] = 0;
        *err = 0;
        return;
    }
    const uint64_t ki = k[i];
    const uint32_t vi = v[i];
    bool d = false;
    for (int w = 1; w <= kResortWindow; ++w) {
        if (i - w >= 0 && !kv_less(k[i - w], v[i - w], ki, vi)) d = true;
        if (i + w < N && !kv_less(ki, vi, k[i + w], v[i + w])) d = true;
    }
    flag[i] = d ? 1 : 0;
}

// split into D (flagged, in order) and R (the rest, in order)
__global__ void k_split_dr(const uint64_t* __restrict__ k, const uint32_t* __restrict__ v, int64_t N,
                           const int* __restrict__ flag, const int* __restrict__ dpos, uint64_t* __restrict__ dk,
                           uint32_t* __restrict__ dv, uint64_t* __restrict__ rk, uint32_t* __restrict__ rv) {
    int64_t i = blockIdx.x * int64_t(TB) + threadIdx.x;
    if (i >= N) return;
    if (flag[i]) {
        dk[dpos[i]] = k[i];
        dv[dpos[i]] = v[i];
    } else {
        const int64_t r = i - dpos[i];
        rk[r] = k[i];
        rv[r] = v[i];
    }
}

// err |= 1 when R (size N - dpos[N]) is not sorted
__global__ void k_check_sorted(const uint64_t* __restrict__ rk, const uint32_t* __restrict__ rv, int64_t N,
                               const int* __restrict__ dpos, int* __restrict__ err) {
    int64_t r = blockIdx.x * int64_t(TB) + threadIdx.x;
    const int64_t nr = N - dpos[N];
    if (r + 1 >= nr) return;
    if (!kv_less(rk[r], rv[r], rk[r + 1], rv[r + 1])) atomicOr(err, 1);
}

// after a stable sort of D by key: runs of equal keys put in index order
__global__ void k_fix_ties(const uint64_t* __restrict__ dk, uint32_t* __restrict__ dv, int64_t n) {
    int64_t i = blockIdx.x * int64_t(TB) + threadIdx.x;
    if (i >= n || (i > 0 && dk[i - 1] == dk[i])) return;
    int64_t e = i + 1;
    while (e < n && dk[e] == dk[i]) ++e;
    for (int64_t a = i + 1; a < e; ++a) {   // insertion sort of the (short) run
        const uint32_t t = dv[a];
        int64_t b = a;
        while (b > i && dv[b - 1] > t) {
            dv[b] = dv[b - 1];
            --b;
        }
        dv[b] = t;
    }
}

// number of elements of the sorted (k, v)[0, n) before (key, val)
__device__ inline int64_t rank_in(const uint64_t* __restrict__ k, const uint32_t* __restrict__ v, int64_t n,
                                  uint64_t key, uint32_t val) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (kv_less(k[mid], v[mid], key, val)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// merge: every element of A goes to its index plus its rank in B
__global__ void k_merge_into(const uint64_t* __restrict__ ak, const uint32_t* __restrict__ av, int64_t na,
                             const uint64_t* __restrict__ bk, const uint32_t* __restrict__ bv, int64_t nb,
                             uint64_t* __restrict__ ok, uint32_t* __restrict__ ov) {
    int64_t i = blockIdx.x * int64_t(TB) + threadIdx.x;
    if (i >= na) return;
    const int64_t p = i + rank_in(bk, bv, nb, ak[i], av[i]);
    ok[p] = ak[i];
    ov[p] = av[i];
}

// ----------------------------------------------------------------- scan
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = TB * SCAN_ITEMS;

template <class T>
__device__ T block_exclusive_scan(T v, T* total) {
    __shared__ T sh[TB];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < TB; off <<= 1) {
        T t = threadIdx.x >= off ? sh[threadIdx.x - off] : T(0);
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    T incl = sh[threadIdx.x];
    *total = sh[TB - 1];
    __syncthreads();
    return incl - v;
}

template <class T>
__global__ void k_scan_tiles(const T* __restrict__ in, T* __restrict__ out, int64_t n, T* __restrict__ sums) {
    int64_t base = blockIdx.x * int64_t(SCAN_TILE) + threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    T run = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = base + k < n ? in[base + k] : T(0);
        T t = v[k];
        v[k] = run;
        run += t;
    }
    T total;
    T off = block_exclusive_scan<T>(run, &total);
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) out[base + k] = v[k] + off;
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <class T>
__global__ void k_scan_add(T* __restrict__ out, int64_t n, const T* __restrict__ sums) {
    int64_t base = blockIdx.x * int64_t(SCAN_TILE) + threadIdx.x * SCAN_ITEMS;
    T a = sums[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) out[base + k] += a;
}

// Exclusive scan of at most SCAN_ONE values in one block of 1,024 threads
// (one launch): thread t scans its run of 16 in registers, the run totals are
// scanned across the wave by shuffles and across the 16 waves in LDS.
constexpr int SCAN_ONE_THREADS = 1024, SCAN_ONE_ITEMS = 16;
constexpr int SCAN_ONE = SCAN_ONE_THREADS * SCAN_ONE_ITEMS;   // 16384 values
template <class T>
__device__ inline void scan_one_body(const T* __restrict__ in, T* __restrict__ out, T* __restrict__ out2, int n) {
    __shared__ T wsum[SCAN_ONE_THREADS / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int base = t * SCAN_ONE_ITEMS;
    T v[SCAN_ONE_ITEMS];
    T run = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ONE_ITEMS; ++k) {
        const T x = base + k < n ? in[base + k] : T(0);
        v[k] = run;
        run += x;
    }
    T incl = run;   // inclusive scan of the run totals within the wave
    for (int d = 1; d < 64; d <<= 1) {
        const T y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    if (w == 0) {
        T x = lane < SCAN_ONE_THREADS / 64 ? wsum[lane] : T(0);
        for (int d = 1; d < 16; d <<= 1) {
            const T y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane < SCAN_ONE_THREADS / 64) wsum[lane] = x;   // inclusive over the waves
    }
    __syncthreads();
    const T off = (incl - run) + (w > 0 ? wsum[w - 1] : T(0));
#pragma unroll
    for (int k = 0; k < SCAN_ONE_ITEMS; ++k)
        if (base + k < n) {
            out[base + k] = v[k] + off;
            if (out2) out2[base + k] = v[k] + off;
        }
}

template <class T>
__global__ __launch_bounds__(SCAN_ONE_THREADS) void k_scan_one(const T* __restrict__ in, T* __restrict__ out, int n) {
    scan_one_body<T>(in, out, nullptr, n);
}

// Two independent scans of at most SCAN_ONE values, one block each; the first
// may also write a copy of its result (out2, nullable).
template <class T>
__global__ __launch_bounds__(SCAN_ONE_THREADS) void k_scan_one2(const T* __restrict__ in0, T* __restrict__ out0,
                                                                T* __restrict__ copy0, int n0,
                                                                const T* __restrict__ in1, T* __restrict__ out1,
                                                                int n1) {
    if (blockIdx.x == 0) scan_one_body<T>(in0, out0, copy0, n0);
    else scan_one_body<T>(in1, out1, nullptr, n1);
}

// Exclusive scan of n values (in may equal out).  The tile sums of nested
// levels live in four equal slabs of P->scan_tmp, sized at the top level.
template <class T>
void exclusive_scan(kifmm_plan* P, const T* in, T* out, int64_t n, hipStream_t s, int depth = 0) {
    if (n <= 0) return;
    if (depth == 0 && n > SCAN_TILE && n <= SCAN_ONE) {
        hipLaunchKernelGGL(k_scan_one<T>, dim3(1), dim3(SCAN_ONE_THREADS), 0, s, in, out, int(n));
        return;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (depth == 0) P->scan_tmp.ensure(4 * (size_t(nb) * 8 + 256));
    if (depth >= 4) throw Error(KIFMM_ERR_STATE, "scan too deep");
    size_t slab = (P->scan_tmp.cap / 4) & ~size_t(255);
    T* sums = reinterpret_cast<T*>(P->scan_tmp.as<char>() + size_t(depth) * slab);
    hipLaunchKernelGGL(k_scan_tiles<T>, dim3(unsigned(nb)), dim3(TB), 0, s, in, out, n, sums);
    if (nb > 1) {
        exclusive_scan<T>(P, sums, sums, nb, s, depth + 1);
        hipLaunchKernelGGL(k_scan_add<T>, dim3(unsigned(nb)), dim3(TB), 0, s, out, n, sums);
    }
}

template <class T>
__global__ void k_copy_int_t(const T* __restrict__ a, T* __restrict__ b, int64_t n) {
    const int64_t i = blockIdx.x * int64_t(TB) + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// Two exclusive scans (in may equal out), in one launch when both fit one
// block; copy0 (nullable) receives a copy of the first result; n1 = 0 scans
// only the first.
template <class T>
void exclusive_scan2(kifmm_plan* P, const T* in0, T* out0, T* copy0, int64_t n0, const T* in1, T* out1, int64_t n1,
                     hipStream_t s) {
    if (n0 <= SCAN_ONE && n1 <= SCAN_ONE && n0 > 0) {
        hipLaunchKernelGGL(k_scan_one2<T>, dim3(n1 > 0 ? 2 : 1), dim3(SCAN_ONE_THREADS), 0, s, in0, out0, copy0,
                           int(n0), in1, out1, int(n1));
        return;
    }
    exclusive_scan<T>(P, in0, out0, n0, s);
    if (copy0 && n0 > 0) hipLaunchKernelGGL(k_copy_int_t<T>, dim3(nblocks(n0)), dim3(TB), 0, s, out0, copy0, n0);
    exclusive_scan<T>(P, in1, out1, n1, s);
}

// ----------------------------------------------------------------- radix sort
constexpr int RS_ITEMS = 16;
constexpr int RS_WAVE_ITEMS = 64 * RS_ITEMS;   // 1024 keys per wave
constexpr int RS_TILE = 4 * RS_WAVE_ITEMS;     // 4096 keys per block

__global__ void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                          uint32_t* __restrict__ hist, int nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = blockIdx.x * int64_t(RS_TILE);
    for (int k = threadIdx.x; k < RS_TILE; k += TB) {
        int64_t i = base + k;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[int64_t(threadIdx.x) * nblk + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: wave w owns the contiguous quarter [w*1024, (w+1)*1024) of
// the block's tile and walks it in 16 rounds of 64 keys; peers with equal
// digits are found with eight ballots, so ranks follow the input order.
__global__ __launch_bounds__(256) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                    const uint32_t* __restrict__ vin,
                                                    uint64_t* __restrict__ kout,
                                                    uint32_t* __restrict__ vout, int64_t n, int shift,
                                                    const uint32_t* __restrict__ off, int nblk) {
    __shared__ uint32_t cnt[4][256];
    __shared__ uint32_t base[4][256];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t b0 = blockIdx.x * int64_t(RS_TILE) + w * int64_t(RS_WAVE_ITEMS);
    uint64_t k[RS_ITEMS];
    uint32_t v[RS_ITEMS];
    for (int r = 0; r < RS_ITEMS; ++r) {
        int64_t i = b0 + r * 64 + lane;
        k[r] = i < n ? kin[i] : 0;
        v[r] = i < n ? vin[i] : 0;
    }
    for (int d = threadIdx.x; d < 4 * 256; d += TB) (&cnt[0][0])[d] = 0;
    __syncthreads();
    const uint64_t lt = lane_lt_mask();
    for (int r = 0; r < RS_ITEMS; ++r) {
        int64_t i = b0 + r * 64 + lane;
        bool valid = i < n;
        uint32_t dg = uint32_t(k[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
        for (int bt = 0; bt < 8; ++bt) {
            uint64_t m = __ballot((dg >> bt) & 1u);
            peers &= ((dg >> bt) & 1u) ? m : ~m;
        }
        if (valid && (peers & lt) == 0) cnt[w][dg] += uint32_t(__popcll(peers));
    }
    __syncthreads();
    {
        int d = threadIdx.x;
        uint32_t run = off[int64_t(d) * nblk + blockIdx.x];
        for (int ww = 0; ww < 4; ++ww) {
            base[ww][d] = run;
            run += cnt[ww][d];
        }
    }
    __syncthreads();
    for (int r = 0; r < RS_ITEMS; ++r) {
        int64_t i = b0 + r * 64 + lane;
        bool valid = i < n;
        uint32_t dg = uint32_t(k[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
        for (int bt = 0; bt < 8; ++bt) {
            uint64_t m = __ballot((dg >> bt) & 1u);
            peers &= ((dg >> bt) & 1u) ? m : ~m;
        }
        uint32_t pos = 0;
        if (valid) pos = base[w][dg] + uint32_t(__popcll(peers & lt));
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            kout[pos] = k[r];
            vout[pos] = v[r];
            if ((peers & lt) == 0) base[w][dg] += uint32_t(__popcll(peers));
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Keys per wave when n keys are dealt to nw waves in contiguous runs of whole
// rounds of 64 (at most RS_WAVE_ITEMS): a small sort takes only the rounds
// it needs, on every wave alike.
__device__ inline int rs_chunk(int n, int nw) { return ((n + 64 * nw - 1) / (64 * nw)) * 64; }

// The whole sort of at most RS_TILE keys in one block: each pass ranks the
// keys as k_rs_scatter does (wave w owns the contiguous run [w*cw, (w+1)*cw),
// peers by ballots), takes the digit offsets from the block's own counts and
// scatters into LDS, from where the next pass reloads its run.
__global__ __launch_bounds__(256) void k_rs_block(uint64_t* __restrict__ keys, uint32_t* __restrict__ vals, int n,
                                                  int passes) {
    __shared__ uint64_t sk[RS_TILE];
    __shared__ uint32_t sv[RS_TILE];
    __shared__ uint32_t cnt[4][256];
    __shared__ uint32_t base[4][256];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cw = rs_chunk(n, 4), nr = cw / 64;
    const int b0 = w * cw;
    uint64_t k[RS_ITEMS];
    uint32_t v[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int i = b0 + r * 64 + lane;
        k[r] = (r < nr && i < n) ? keys[i] : 0;
        v[r] = (r < nr && i < n) ? vals[i] : 0;
    }
    const uint64_t lt = lane_lt_mask();
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = 8 * ps;
        for (int d = threadIdx.x; d < 4 * 256; d += TB) (&cnt[0][0])[d] = 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RS_ITEMS; ++r) {
            if (r < nr) {
                const bool valid = b0 + r * 64 + lane < n;
                const uint32_t dg = uint32_t(k[r] >> shift) & 255u;
                uint64_t peers = __ballot(valid);
                for (int bt = 0; bt < 8; ++bt) {
                    const uint64_t m = __ballot((dg >> bt) & 1u);
                    peers &= ((dg >> bt) & 1u) ? m : ~m;
                }
                if (valid && (peers & lt) == 0) cnt[w][dg] += uint32_t(__popcll(peers));
            }
        }
        __syncthreads();
        {
            // digit-major, then wave: base[w][d] = (keys with a smaller digit)
            // + (keys with digit d in earlier quarters)
            const int d = threadIdx.x;
            const uint32_t t = cnt[0][d] + cnt[1][d] + cnt[2][d] + cnt[3][d];
            uint32_t total;
            uint32_t run = block_exclusive_scan<uint32_t>(t, &total);
            for (int ww = 0; ww < 4; ++ww) {
                base[ww][d] = run;
                run += cnt[ww][d];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RS_ITEMS; ++r) {
            if (r < nr) {
                const bool valid = b0 + r * 64 + lane < n;
                const uint32_t dg = uint32_t(k[r] >> shift) & 255u;
                uint64_t peers = __ballot(valid);
                for (int bt = 0; bt < 8; ++bt) {
                    const uint64_t m = __ballot((dg >> bt) & 1u);
                    peers &= ((dg >> bt) & 1u) ? m : ~m;
                }
                uint32_t pos = 0;
                if (valid) pos = base[w][dg] + uint32_t(__popcll(peers & lt));
                __builtin_amdgcn_wave_barrier();
                if (valid) {
                    sk[pos] = k[r];
                    sv[pos] = v[r];
                    if ((peers & lt) == 0) base[w][dg] += uint32_t(__popcll(peers));
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RS_ITEMS; ++r) {
            const int i = b0 + r * 64 + lane;
            if (r < nr && i < n) {
                k[r] = sk[i];
                v[r] = sv[i];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int i = b0 + r * 64 + lane;
        if (r < nr && i < n) {
            keys[i] = k[r];
            vals[i] = v[r];
        }
    }
}

// The whole sort of at most RS_SMALL keys in one block of RS_SMALL_WAVES
// waves (one launch): wave w holds the run [w cw, (w + 1) cw) in registers,
// ranks them as k_rs_scatter does and scatters each pass into the other of two
// global buffers (keys/vals and ktmp/vtmp), from which the next pass reloads
// its share; an even number of passes ends in keys/vals.
constexpr int kItemOrderMin = 1024;   // leaf work items sorted by cost only above this count
constexpr int RS_SMALL_WAVES = 16;
constexpr int RS_SMALL = RS_SMALL_WAVES * RS_WAVE_ITEMS;   // 16384 keys
__global__ __launch_bounds__(RS_SMALL_WAVES * 64) void k_rs_small(uint64_t* __restrict__ keys,
                                                                  uint32_t* __restrict__ vals,
                                                                  uint64_t* __restrict__ ktmp,
                                                                  uint32_t* __restrict__ vtmp, int n, int passes) {
    __shared__ uint32_t cnt[RS_SMALL_WAVES][256];
    __shared__ uint32_t scan[256];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, t = threadIdx.x;
    const int cw = rs_chunk(n, RS_SMALL_WAVES), nr = cw / 64;
    const int b0 = w * cw;
    uint64_t k[RS_ITEMS];
    uint32_t v[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int i = b0 + r * 64 + lane;
        k[r] = (r < nr && i < n) ? keys[i] : 0;
        v[r] = (r < nr && i < n) ? vals[i] : 0;
    }
    const uint64_t lt = lane_lt_mask();
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = 8 * ps;
        uint64_t* kout = (ps & 1) ? keys : ktmp;
        uint32_t* vout = (ps & 1) ? vals : vtmp;
        for (int d = t; d < RS_SMALL_WAVES * 256; d += RS_SMALL_WAVES * 64) (&cnt[0][0])[d] = 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RS_ITEMS; ++r) {
            if (r < nr) {
                const bool valid = b0 + r * 64 + lane < n;
                const uint32_t dg = uint32_t(k[r] >> shift) & 255u;
                uint64_t peers = __ballot(valid);
                for (int bt = 0; bt < 8; ++bt) {
                    const uint64_t m = __ballot((dg >> bt) & 1u);
                    peers &= ((dg >> bt) & 1u) ? m : ~m;
                }
                if (valid && (peers & lt) == 0) cnt[w][dg] += uint32_t(__popcll(peers));
            }
        }
        __syncthreads();
        // exclusive scan over the digits of the totals, then per wave
        uint32_t tot = 0;
        if (t < 256)
            for (int ww = 0; ww < RS_SMALL_WAVES; ++ww) tot += cnt[ww][t];
        if (t < 256) scan[t] = tot;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const uint32_t a = (t < 256 && t >= off) ? scan[t - off] : 0u;
            __syncthreads();
            if (t < 256) scan[t] += a;
            __syncthreads();
        }
        if (t < 256) {
            uint32_t run = scan[t] - tot;
            for (int ww = 0; ww < RS_SMALL_WAVES; ++ww) {
                const uint32_t c = cnt[ww][t];
                cnt[ww][t] = run;   // becomes the wave's base for digit t
                run += c;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RS_ITEMS; ++r) {
            if (r < nr) {
                const bool valid = b0 + r * 64 + lane < n;
                const uint32_t dg = uint32_t(k[r] >> shift) & 255u;
                uint64_t peers = __ballot(valid);
                for (int bt = 0; bt < 8; ++bt) {
                    const uint64_t m = __ballot((dg >> bt) & 1u);
                    peers &= ((dg >> bt) & 1u) ? m : ~m;
                }
                uint32_t pos = 0;
                if (valid) pos = cnt[w][dg] + uint32_t(__popcll(peers & lt));
                __builtin_amdgcn_wave_barrier();
                if (valid) {
                    kout[pos] = k[r];
                    vout[pos] = v[r];
                    if ((peers & lt) == 0) cnt[w][dg] += uint32_t(__popcll(peers));
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();   // the pass's stores are visible to the whole block
#pragma unroll
        for (int r = 0; r < RS_ITEMS; ++r) {
            const int i = b0 + r * 64 + lane;
            if (r < nr && i < n) {
                k[r] = kout[i];
                v[r] = vout[i];
            }
        }
        __syncthreads();
    }
}

void radix_sort(kifmm_plan* P, uint64_t* keys, uint32_t* vals, uint64_t* ktmp, uint32_t* vtmp, int64_t n,
                int bits, hipStream_t s) {
    if (n <= 0) return;
    const bool even = ((bits + 7) / 8) % 2 == 0;
    // one launch: up to 1,024 keys (or an odd number of passes) four waves
    // exchanging through LDS, else sixteen waves exchanging through L2
    if (n <= RS_TILE && (n <= 1024 || !even)) {
        hipLaunchKernelGGL(k_rs_block, dim3(1), dim3(TB), 0, s, keys, vals, int(n), (bits + 7) / 8);
        return;
    }
    if (n <= RS_SMALL && even) {
        hipLaunchKernelGGL(k_rs_small, dim3(1), dim3(RS_SMALL_WAVES * 64), 0, s, keys, vals, ktmp, vtmp, int(n),
                           (bits + 7) / 8);
        return;
    }
    int nblk = int((n + RS_TILE - 1) / RS_TILE);
    P->tmp_f.ensure(size_t(256) * nblk * 4);
    uint32_t* hist = P->tmp_f.as<uint32_t>();
    uint64_t *ka = keys, *kb = ktmp;
    uint32_t *va = vals, *vb = vtmp;
    int passes = (bits + 7) / 8;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = 8 * ps;
        hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(TB), 0, s, ka, n, shift, hist, nblk);
        exclusive_scan<uint32_t>(P, hist, hist, int64_t(256) * nblk, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(TB), 0, s, ka, va, kb, vb, n, shift, hist, nblk);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        KIFMM_HIP(hipMemcpyAsync(keys, ka, n * 8, hipMemcpyDeviceToDevice, s));
        KIFMM_HIP(hipMemcpyAsync(vals, va, n * 4, hipMemcpyDeviceToDevice, s));
    }
}

// ----------------------------------------------------------------- tree levels
// For each non-leaf parent at level l: child boundaries in its sorted key run
// (the level-(l+1) digit is non-decreasing inside the run).
// One wave per front box.  Lane group g (lanes 9g .. 9g+8, g < 7) finds child
// boundary o = g + 1, the first index of the box's key run whose octant digit
// at level l + 1 is >= o: every step samples 9 points of the group's interval
// and keeps the tenth that holds the boundary (exact once the interval has
// fewer than 10 entries).
// Writes per front box its child count c and non-leaf child count n packed
// as c | n << 32 (and a zero at index nf, so that one exclusive scan of nf + 1
// values gives both offsets).
// One wave: child boundaries of front box f (key run r) at level l; lane 0
// writes the 9 bounds to out and returns the packed counts (others return 0).
__device__ inline unsigned long long split_box(int2 r, int l, const uint64_t* __restrict__ keys, int lane,
                                               int* __restrict__ out, int leaf_size, int adaptive, int max_depth,
                                               int Lu) {
    const int shift = 3 * (kBits - (l + 1));
    const int grp = lane / 9, k = lane % 9;
    const int o = grp + 1;
    int lo = r.x, hi = r.y;   // the boundary lies in [lo, hi]
    // sample j of the interval [lo, lo + len)
    auto sample = [&](int j, int len) -> int { return len >= 10 ? lo + int(int64_t(len) * (j + 1) / 10) : lo + j; };
    while (__ballot(grp < 7 && hi > lo)) {
        const int len = hi - lo;
        const bool act = grp < 7 && len > 0;
        const bool valid = act && (len >= 10 || k < len);
        bool pred = false;
        if (valid) pred = int((keys[sample(k, len)] >> shift) & 7ull) >= o;
        const unsigned long long m = __ballot(pred);
        if (act) {
            const unsigned gm = unsigned(m >> (9 * grp)) & 0x1ffu;
            if (len < 10) {
                lo = gm ? lo + __builtin_ctz(gm) : hi;
                hi = lo;
            } else if (gm) {
                const int ks = __builtin_ctz(gm);
                const int nlo = ks ? sample(ks - 1, len) + 1 : lo;
                hi = sample(ks, len);
                lo = nlo;
            } else {
                lo = sample(8, len) + 1;
            }
        }
    }
    int bd[9];
    bd[0] = r.x;
    bd[8] = r.y;
#pragma unroll
    for (int q = 1; q < 8; ++q) bd[q] = __shfl(lo, 9 * (q - 1), 64);
    if (lane != 0) return 0;
    int c = 0, nl = 0;
    for (int q = 0; q < 9; ++q) out[q] = bd[q];
    for (int q = 0; q < 8; ++q) {
        const int cnt = bd[q + 1] - bd[q];
        if (cnt > 0) {
            ++c;
            const bool leaf = adaptive ? (cnt <= leaf_size || l + 1 == max_depth) : (l + 1 == Lu);
            if (!leaf) ++nl;
        }
    }
    return (unsigned long long)c | ((unsigned long long)nl << 32);
}

__global__ void k_split(const int* __restrict__ front, int nf, int l, const uint64_t* __restrict__ keys,
                        const int2* __restrict__ range, int* __restrict__ bounds /*[nf][9]*/,
                        unsigned long long* __restrict__ cnt, int leaf_size, int adaptive, int max_depth, int Lu) {
    const int64_t gid = int64_t(blockIdx.x) * TB + threadIdx.x;
    const int f = int(gid >> 6), lane = int(gid & 63);
    if (gid == 0) cnt[nf] = 0;
    if (f >= nf) return;   // uniform over the wave
    const unsigned long long c =
        split_box(range[front[f]], l, keys, lane, bounds + 9 * f, leaf_size, adaptive, max_depth, Lu);
    if (lane == 0) cnt[f] = c;
}

// Eight lanes per front box, lane o writing child octant o: a child's index
// and its place in the non-leaf list are the counts of the non-empty (and
// non-leaf) octants below it, so the children keep the octant order.  The
// eight lanes of a box are lanes 8k .. 8k+7 of one wave; every lane of the
// wave calls this (act = false for lanes without a box).
__device__ inline void emit_box(bool act, int f, int o, int l, const int* __restrict__ front,
                                const uint64_t* __restrict__ keys, const int* __restrict__ bounds,
                                const unsigned long long* __restrict__ off, int child_start, int nl_base,
                                int4* __restrict__ anchor, int2* __restrict__ range, int* __restrict__ parent,
                                int2* __restrict__ child, int* __restrict__ leafflag, uint64_t* __restrict__ mkey,
                                int* __restrict__ nonleaf, int leaf_size, int adaptive, int max_depth, int Lu) {
    int cnt = 0, b0 = 0, b1 = 0;
    if (act) {
        const int* bd = bounds + 9 * f;
        b0 = bd[o];
        b1 = bd[o + 1];
        cnt = b1 - b0;
    }
    const bool has = act && cnt > 0;
    const bool leaf = adaptive ? (cnt <= leaf_size || l + 1 == max_depth) : (l + 1 == Lu);
    const bool inner = has && !leaf;
    const int sh8 = (threadIdx.x & 63) & ~7;   // this box's 8 lanes within the wave
    const unsigned mh = unsigned(__ballot(has) >> sh8) & 0xffu;
    const unsigned mn = unsigned(__ballot(inner) >> sh8) & 0xffu;
    if (!act) return;
    const int P = front[f];
    const unsigned long long of = off[f];   // child offset | non-leaf offset << 32
    const int first = child_start + int(of & 0xffffffffull);
    const unsigned below = (1u << o) - 1u;
    if (has) {
        const int c = first + __popc(mh & below);
        const int4 a = anchor[P];
        anchor[c] = make_int4(2 * a.x + ((o >> 2) & 1), 2 * a.y + ((o >> 1) & 1), 2 * a.z + (o & 1), l + 1);
        range[c] = make_int2(b0, b1);
        parent[c] = P;
        child[c] = make_int2(-1, 0);
        leafflag[c] = leaf ? 1 : 0;
        mkey[c] = keys[b0] >> (3 * (kBits - (l + 1)));
        if (inner) nonleaf[nl_base + int(of >> 32) + __popc(mn & below)] = c;
    }
    if (o == 0) child[P] = make_int2(first, int(mh));
}

__global__ void k_emit(const int* __restrict__ front, int nf, int l, const uint64_t* __restrict__ keys,
                       const int* __restrict__ bounds, const unsigned long long* __restrict__ off,
                       int child_start, int nl_base,
                       int4* __restrict__ anchor, int2* __restrict__ range, int* __restrict__ parent,
                       int2* __restrict__ child, int* __restrict__ leafflag, uint64_t* __restrict__ mkey,
                       int* __restrict__ nonleaf, int leaf_size, int adaptive, int max_depth, int Lu) {
    const int64_t gid = int64_t(blockIdx.x) * TB + threadIdx.x;
    const int f = int(gid >> 3), o = int(gid & 7);
    emit_box(f < nf, f, o, l, front, keys, bounds, off, child_start, nl_base, anchor, range, parent, child, leafflag,
             mkey, nonleaf, leaf_size, adaptive, max_depth, Lu);
}

// Every level of a small tree in one block (one launch, no read-back per
// level): per level, split the front boxes (one wave each), scan their child
// counts, emit the children.  lev[l] = (start, count, nl_start, nl_count);
// lev_n[0] = number of levels, lev_n[1] = 1 when the box storage `cap` or the
// scratch (nf_cap front boxes) would overflow, then the caller builds the
// levels the general way.
constexpr int LB_THREADS = 1024;
__global__ __launch_bounds__(LB_THREADS) void k_levels_block(
    const uint64_t* __restrict__ keys, int cap, int nf_cap, int* __restrict__ bounds,
    unsigned long long* __restrict__ cnt, unsigned long long* __restrict__ off, int4* __restrict__ anchor,
    int2* __restrict__ range, int* __restrict__ parent, int2* __restrict__ child, int* __restrict__ leafflag,
    uint64_t* __restrict__ mkey, int* __restrict__ nonleaf, int4* __restrict__ lev, int* __restrict__ lev_n,
    int leaf_size, int adaptive, int max_depth, int Lu, int root_nl, int N) {
    __shared__ unsigned long long wsum[LB_THREADS / 64];
    __shared__ unsigned long long carry;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = LB_THREADS / 64;
    int start = 0, count = 1, nl_start = 0, nl_count = root_nl;
    int total = 1, nl_total = root_nl;
    if (t == 0) {
        // the root box (a non-leaf here), as k_root writes it for the general build
        anchor[0] = make_int4(0, 0, 0, 0);
        range[0] = make_int2(0, N);
        parent[0] = -1;
        child[0] = make_int2(-1, 0);
        leafflag[0] = 0;
        mkey[0] = 0;
        nonleaf[0] = 0;
        lev[0] = make_int4(0, 1, 0, root_nl);
        lev_n[1] = 0;
    }
    __syncthreads();
    int l = 0;
    for (; nl_count > 0; ++l) {
        if (l + 1 >= kMaxLevels || nl_count > nf_cap) {
            if (t == 0) lev_n[1] = 1;
            break;
        }
        const int nf = nl_count;
        const int* front = nonleaf + nl_start;
        // split: one wave per front box
        for (int f = wave; f < nf; f += nw) {
            const unsigned long long c =
                split_box(range[front[f]], l, keys, lane, bounds + 9 * f, leaf_size, adaptive, max_depth, Lu);
            if (lane == 0) cnt[f] = c;
        }
        __syncthreads();
        // exclusive scan of the packed counts (chunks of LB_THREADS, in order)
        if (t == 0) carry = 0;
        __syncthreads();
        for (int c0 = 0; c0 < nf; c0 += LB_THREADS) {
            const int i = c0 + t;
            const unsigned long long v = i < nf ? cnt[i] : 0ull;
            unsigned long long x = v;   // inclusive scan within the wave
            for (int d = 1; d < 64; d <<= 1) {
                const unsigned long long y = __shfl_up(x, d, 64);
                if (lane >= d) x += y;
            }
            if (lane == 63) wsum[wave] = x;
            __syncthreads();
            if (t == 0) {
                unsigned long long a = carry;
                for (int w = 0; w < nw; ++w) {
                    const unsigned long long b = wsum[w];
                    wsum[w] = a;
                    a += b;
                }
                carry = a;
            }
            __syncthreads();
            if (i < nf) off[i] = wsum[wave] + x - v;
            __syncthreads();
        }
        const unsigned long long tot = carry;
        const int ncount = int(tot & 0xffffffffull), nnl = int(tot >> 32);
        if (total + ncount > cap) {
            if (t == 0) lev_n[1] = 1;
            break;
        }
        __syncthreads();
        // emit: eight lanes per front box
        for (int g0 = 0; g0 < nf * 8; g0 += LB_THREADS) {
            const int gid = g0 + t;
            const int f = gid >> 3, o = gid & 7;
            emit_box(f < nf, f, o, l, front, keys, bounds, off, total, nl_total, anchor, range, parent, child,
                     leafflag, mkey, nonleaf, leaf_size, adaptive, max_depth, Lu);
        }
        __syncthreads();
        start = total;
        count = ncount;
        nl_start = nl_total;
        nl_count = nnl;
        total += ncount;
        nl_total += nnl;
        if (t == 0) lev[l + 1] = make_int4(start, count, nl_start, nl_count);
    }
    if (t == 0) lev_n[0] = l + 1;
}

__global__ void k_root(int N, int leaf, int4* anchor, int2* range, int* parent, int2* child, int* leafflag,
                       uint64_t* mkey, int* nonleaf) {
    anchor[0] = make_int4(0, 0, 0, 0);
    range[0] = make_int2(0, N);
    parent[0] = -1;
    child[0] = make_int2(-1, 0);
    leafflag[0] = leaf;
    mkey[0] = 0;
    if (!leaf) nonleaf[0] = 0;
}

__global__ void k_gather_pos(const double* __restrict__ x, const uint32_t* __restrict__ idx, int64_t N,
                             float4* __restrict__ xs, int* __restrict__ perm) {
    int64_t i = blockIdx.x * int64_t(TB) + threadIdx.x;
    if (i >= N) return;
    uint32_t j = idx[i];
    xs[i] = make_float4(float(x[3 * size_t(j)]), float(x[3 * size_t(j) + 1]), float(x[3 * size_t(j) + 2]), 0.f);
    perm[i] = int(j);
}

// ----------------------------------------------------------------- lists
// Closed cubes on the finest integer grid touch or overlap: box b and the
// image of box a that list entry e names (shifted by whole root widths).
__device__ inline bool adjacent_image(int4 a, int e, int4 b) {
    int sx, sy, sz;
    img_shift(e, sx, sy, sz);
    const int L = 1 << kBits;
    int sa = kBits - a.w, sb = kBits - b.w;
    int ax0 = (a.x << sa) + sx * L, ay0 = (a.y << sa) + sy * L, az0 = (a.z << sa) + sz * L, ea = 1 << sa;
    int bx0 = b.x << sb, by0 = b.y << sb, bz0 = b.z << sb, eb = 1 << sb;
    return ax0 <= bx0 + eb && bx0 <= ax0 + ea && ay0 <= by0 + eb && by0 <= ay0 + ea && az0 <= bz0 + eb &&
           bz0 <= az0 + ea;
}

__device__ inline int find_box(const uint64_t* __restrict__ mkey, int start, int count, uint64_t key) {
    int lo = start, hi = start + count;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (mkey[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < start + count && mkey[lo] == key) ? lo : -1;
}

// One thread per (box, direction): a binary search for the neighbour's key
// among the boxes of the same level.  Periodic: the neighbour cell wraps
// around the root and the entry records the image shift.
__global__ void k_colleagues(int B, const int4* __restrict__ anchor, const uint64_t* __restrict__ mkey,
                             LevelTable lt, int periodic, int* __restrict__ coll) {
    const int64_t g = int64_t(blockIdx.x) * TB + threadIdx.x;
    if (g >= int64_t(B) * 27) return;
    const int b = int(g / 27), d = int(g % 27);
    const int4 a = anchor[b];
    const int l = a.w;
    const int lim = 1 << l;
    int x = a.x + d / 9 - 1, y = a.y + (d / 3) % 3 - 1, z = a.z + d % 3 - 1;
    int id = -1;
    if (periodic) {
        const int sx = x < 0 ? -1 : (x >= lim ? 1 : 0);
        const int sy = y < 0 ? -1 : (y >= lim ? 1 : 0);
        const int sz = z < 0 ? -1 : (z >= lim ? 1 : 0);
        x -= sx * lim;
        y -= sy * lim;
        z -= sz * lim;
        const int f = find_box(mkey, lt.start[l], lt.count[l], morton3(x, y, z));
        if (f >= 0) id = img_encode(f, sx, sy, sz);
    } else if (x >= 0 && y >= 0 && z >= 0 && x < lim && y < lim && z < lim) {
        id = find_box(mkey, lt.start[l], lt.count[l], morton3(x, y, z));
    }
    coll[g] = id;
}

// V-list slots of an octant: (colleague direction D in 0..26, child octant o')
// pairs whose offset d = 2 (D - 1) + o' - o is not adjacent, ordered by the
// lexicographic index of d among the 316 far offsets.
struct VTable {
    unsigned char D[8][kVPerOct];
    unsigned char oc[8][kVPerOct];
    short op[8][kVPerOct];
};

// One wave per box, the lanes over its 189 slots (coalesced rows).
__global__ void k_vdense(int b0, int nb, const int4* __restrict__ anchor, const int* __restrict__ parent,
                         const int2* __restrict__ child, const int* __restrict__ leafflag,
                         const int* __restrict__ coll, const VTable* __restrict__ vt, int* __restrict__ vd) {
    const int64_t g = int64_t(blockIdx.x) * TB + threadIdx.x;
    const int i = int(g >> 6), lane = int(g & 63);
    if (i >= nb) return;
    const int b = b0 + i;
    const int4 a = anchor[b];
    const int o = ((a.x & 1) << 2) | ((a.y & 1) << 1) | (a.z & 1);
    int* out = vd + int64_t(i) * kVPerOct;
    if (parent[b] < 0) {   // the (periodic) root: no V list
        for (int j = lane; j < kVPerOct; j += 64) out[j] = -1;
        return;
    }
    const int* cp = coll + 27 * int64_t(parent[b]);
    for (int j = lane; j < kVPerOct; j += 64) {
        // the slot fixes the offset; an image's shift needs no record
        const int Qe = cp[vt->D[o][j]];
        const int Q = Qe >= 0 ? img_box(Qe) : -1;
        int src = -1;
        if (Q >= 0 && !leafflag[Q]) {
            const int2 c = child[Q];
            const int oc = vt->oc[o][j];
            if ((c.y >> oc) & 1) src = c.x + __popc(c.y & ((1 << oc) - 1));
        }
        out[j] = src;
    }
}

// The next three kernels take one wave per box.  Its candidates are the 27
// colleagues of a box P (lanes 0..26) and, when P has them, P's coarse
// adjacent leaves (lanes 27..52, a row that ends at its first -1); each lane
// tests its own candidate and the kept ones are compacted in lane order by a
// ballot, which is the order of a serial walk over the two rows.
__device__ inline int wave_candidate(int lane, int P, bool with_cal, const int* __restrict__ coll,
                                     const int* __restrict__ cal) {
    if (lane < 27) return coll[27 * int64_t(P) + lane];
    if (with_cal && lane < 53) return cal[26 * int64_t(P) + (lane - 27)];
    return -1;
}

// Coarse adjacent leaves: leaves of a coarser level adjacent to b; at most 26.
// They are the leaf colleagues of parent(b) and the coarse adjacent leaves of
// parent(b) that touch b.
__global__ __launch_bounds__(256) void k_cal(int b0, int nb, const int4* __restrict__ anchor,
                                             const int* __restrict__ parent, const int* __restrict__ leafflag,
                                             const int* __restrict__ coll, int* __restrict__ cal,
                                             int* __restrict__ bad) {
    const int lane = threadIdx.x & 63, i = blockIdx.x * 4 + int(threadIdx.x >> 6);
    if (i >= nb) return;   // whole wave
    const int b = b0 + i;
    const int4 ab = anchor[b];
    const int P = parent[b];
    // (the root has no coarse adjacent leaves; its row is never written)
    const int Q = wave_candidate(lane, P, P > 0, coll, cal);
    bool keep = false;
    if (Q >= 0) {
        const int A = img_box(Q);
        keep = (lane >= 27 || leafflag[A]) && adjacent_image(anchor[A], Q, ab);
    }
    const uint64_t m = __ballot(keep);
    const int cnt = __popcll(m), pos = __popcll(m & lane_lt_mask());
    int* out = cal + 26 * int64_t(b);
    if (keep && pos < 26) out[pos] = Q;
    if (lane >= cnt && lane < 26) out[lane] = -1;
    if (lane == 0 && cnt > 26) atomicOr(bad, 2);
}

// X(b), level >= 2: leaves adjacent to parent(b) of its level or coarser that
// are not adjacent to b.  mode 0 counts, mode 1 fills.
// The list bodies below take the block index `vb` as an argument, so that
// independent passes can share one launch (the fused kernels further down);
// each wave handles one box and returns on its own (no block barriers).
__device__ inline void xlist_body(int vb, int b0, int nb, const int4* __restrict__ anchor,
                                  const int* __restrict__ parent, const int* __restrict__ leafflag,
                                  const int* __restrict__ coll, const int* __restrict__ cal,
                                  int* __restrict__ cnt_or_off, int* __restrict__ idx, int mode) {
    const int lane = threadIdx.x & 63, i = vb * 4 + int(threadIdx.x >> 6);
    if (i >= nb) return;   // whole wave
    const int b = b0 + i;
    const int P = parent[b];
    if (P < 0) {   // the (periodic) root
        if (!mode && lane == 0) cnt_or_off[b] = 0;
        return;
    }
    const int4 ab = anchor[b];
    const int Q = wave_candidate(lane, P, P > 0, coll, cal);
    bool keep = false;
    if (Q >= 0) {
        const int A = img_box(Q);
        keep = (lane >= 27 || leafflag[A]) && !adjacent_image(anchor[A], Q, ab);
    }
    const uint64_t m = __ballot(keep);
    if (mode) {
        if (keep) idx[cnt_or_off[b] + __popcll(m & lane_lt_mask())] = Q;
    } else if (lane == 0) {
        cnt_or_off[b] = __popcll(m);
    }
}

// U(b) own part: leaf colleagues (b included) and coarse adjacent leaves.
// The count is added (the finer part's count may run in the same launch).
__device__ inline void ulist_own_body(int vb, int B, const int* __restrict__ leafflag,
                                      const int* __restrict__ coll, const int* __restrict__ cal,
                                      int* __restrict__ cnt_or_off, int* __restrict__ idx,
                                      int* __restrict__ cursor, int mode) {
    const int lane = threadIdx.x & 63, b = vb * 4 + int(threadIdx.x >> 6);
    if (b >= B || !leafflag[b]) return;   // whole wave
    const int Q = wave_candidate(lane, b, b > 0, coll, cal);
    const bool keep = Q >= 0 && (lane >= 27 || leafflag[img_box(Q)]);
    const uint64_t m = __ballot(keep);
    const int c = __popcll(m);
    if (mode) {
        const int at = cnt_or_off[b];
        if (keep) idx[at + __popcll(m & lane_lt_mask())] = Q;
        if (lane == 0) cursor[b] = at + c;
    } else if (lane == 0) {
        atomicAdd(&cnt_or_off[b], c);
    }
}

// U(b) finer part: every leaf A lists b in cal[A]  ->  A in U(b) (an image
// of b seen from A is A seen from b with the shift negated).  One wave per
// leaf A, one lane per cal entry (the row sort undoes the atomics' order).
__device__ inline void ulist_fine_body(int vb, int B, const int* __restrict__ leafflag,
                                       const int* __restrict__ cal, int* __restrict__ cnt,
                                       int* __restrict__ idx, int* __restrict__ cursor, int mode) {
    const int lane = threadIdx.x & 63, a = vb * 4 + int(threadIdx.x >> 6);
    if (a >= B || a == 0 || !leafflag[a] || lane >= 26) return;   // a root leaf has no coarse adjacent leaves
    const int e = cal[26 * int64_t(a) + lane];
    if (e < 0) return;   // the row ends at its first -1
    const int b = img_box(e);
    if (mode) idx[atomicAdd(&cursor[b], 1)] = img_flip((e & ~kBoxMask) | a);
    else atomicAdd(&cnt[b], 1);
}

// W(b) = {A : b in X(A)}.  One wave per box A, one lane per X(A) entry (the
// order the atomics give is undone by the row sort).
__device__ inline void wlist_body(int vb, int b0, int nb, const int* __restrict__ xoff,
                                  const int* __restrict__ xidx, int* __restrict__ cnt,
                                  int* __restrict__ idx, int* __restrict__ cursor, int mode) {
    const int lane = threadIdx.x & 63, i = vb * 4 + int(threadIdx.x >> 6);
    if (i >= nb) return;
    const int A = b0 + i;
    for (int k = xoff[A] + lane; k < xoff[A + 1]; k += 64) {
        const int e = xidx[k];
        const int b = img_box(e);
        if (mode) idx[atomicAdd(&cursor[b], 1)] = img_flip((e & ~kBoxMask) | A);
        else atomicAdd(&cnt[b], 1);
    }
}

// Inputs shared by the fused list passes.
struct ListArgs {
    int b2, nvb, B;
    const int4* anchor;
    const int* parent;
    const int* leafflag;
    const int* coll;
    const int* cal;
    int* xoff;
    int* xidx;
    int* uoff;
    int* uidx;
    int* woff;
    int* widx;
    int* cursor;
};

// Counts of X, of the own part of U and of its finer part: three passes over
// disjoint block ranges of one launch (nbx blocks for X, nbu for each U part).
__global__ __launch_bounds__(256) void k_list_counts(ListArgs a, int nbx, int nbu) {
    const int vb = blockIdx.x;
    if (vb < nbx)
        xlist_body(vb, a.b2, a.nvb, a.anchor, a.parent, a.leafflag, a.coll, a.cal, a.xoff, nullptr, 0);
    else if (vb < nbx + nbu)
        ulist_own_body(vb - nbx, a.B, a.leafflag, a.coll, a.cal, a.uoff, nullptr, nullptr, 0);
    else
        ulist_fine_body(vb - nbx - nbu, a.B, a.leafflag, a.cal, a.uoff, nullptr, nullptr, 0);
}

// X entries and the own part of U (which sets the cursor of the finer part).
__global__ __launch_bounds__(256) void k_list_fill_a(ListArgs a, int nbx) {
    const int vb = blockIdx.x;
    if (vb < nbx)
        xlist_body(vb, a.b2, a.nvb, a.anchor, a.parent, a.leafflag, a.coll, a.cal, a.xoff, a.xidx, 1);
    else
        ulist_own_body(vb - nbx, a.B, a.leafflag, a.coll, a.cal, a.uoff, a.uidx, a.cursor, 1);
}

// The finer part of U (from the cursor) and the W counts (from the X lists).
__global__ __launch_bounds__(256) void k_list_fill_b(ListArgs a, int nbu) {
    const int vb = blockIdx.x;
    if (vb < nbu)
        ulist_fine_body(vb, a.B, a.leafflag, a.cal, nullptr, a.uidx, a.cursor, 1);
    else
        wlist_body(vb - nbu, a.b2, a.nvb, a.xoff, a.xidx, a.woff, nullptr, nullptr, 0);
}

// W entries (from the cursor, a copy of the W offsets).
__global__ __launch_bounds__(256) void k_list_fill_w(ListArgs a) {
    wlist_body(blockIdx.x, a.b2, a.nvb, a.xoff, a.xidx, nullptr, a.widx, a.cursor, 1);
}

// Sort each CSR row ascending (entries of a row are distinct).  One wave per
// row: rows of up to SORT_CAP entries are placed by rank (the number of
// smaller entries) through LDS; longer rows fall back to one lane.
constexpr int SORT_CAP = 1024;

// blockIdx.y picks one of up to three lists (offsets, entries), sorted in one launch.
__global__ __launch_bounds__(64) void k_sort_rows(int B, const int* __restrict__ off0, int* __restrict__ idx0,
                                                  const int* __restrict__ off1, int* __restrict__ idx1,
                                                  const int* __restrict__ off2, int* __restrict__ idx2) {
    __shared__ int v[SORT_CAP];
    const int b = blockIdx.x;
    const int* off = blockIdx.y == 0 ? off0 : blockIdx.y == 1 ? off1 : off2;
    int* idx = blockIdx.y == 0 ? idx0 : blockIdx.y == 1 ? idx1 : idx2;
    const int s = off[b], e = off[b + 1], len = e - s;
    if (len <= 1) return;
    if (len <= SORT_CAP) {
        for (int k = threadIdx.x; k < len; k += 64) v[k] = idx[s + k];
        __syncthreads();
        for (int k = threadIdx.x; k < len; k += 64) {
            const int x = v[k];
            int rank = 0;
            for (int m = 0; m < len; ++m) rank += v[m] < x;
            idx[s + rank] = x;
        }
    } else if (threadIdx.x == 0) {
        for (int i = s + 1; i < e; ++i) {
            int x = idx[i];
            int j = i - 1;
            while (j >= s && idx[j] > x) {
                idx[j + 1] = idx[j];
                --j;
            }
            idx[j + 1] = x;
        }
    }
}

// A W/X pair (box A, finer box F: F in W(A), A in X(F)) is summed point to
// point in both directions when F is a leaf with at most n points; those
// pairs join the U list in the near list of each leaf.
__device__ inline bool direct_xw(int f, const int* __restrict__ leafflag, const int2* __restrict__ range, int n) {
    const int2 r = range[f];
    return leafflag[f] && r.y - r.x <= n;
}

// Near list of leaf b: U(b), then X(b) when b is itself such an F, then the
// W(b) boxes that are; and the far W list: the other W(b) boxes.  One wave per
// box, entries copied 64 at a time, the W split kept in order by ballots.
// mode 0 counts (entry B of both count arrays is the scans' last), mode 1 fills.
__global__ __launch_bounds__(256) void k_near(int B, int n, const int* __restrict__ leafflag,
                                              const int2* __restrict__ range, const int* __restrict__ uoff,
                                              const int* __restrict__ uidx, const int* __restrict__ xoff,
                                              const int* __restrict__ xidx, const int* __restrict__ woff,
                                              const int* __restrict__ widx, int* __restrict__ noff,
                                              int* __restrict__ nidx, int* __restrict__ wfoff,
                                              int* __restrict__ wfidx, int mode) {
    const int lane = threadIdx.x & 63, b = blockIdx.x * 4 + int(threadIdx.x >> 6);
    if (b == B && !mode && lane == 0) noff[B] = wfoff[B] = 0;
    if (b >= B) return;   // whole wave
    if (!leafflag[b]) {
        if (!mode && lane == 0) noff[b] = wfoff[b] = 0;
        return;
    }
    const int u0 = uoff[b], nu = uoff[b + 1] - u0;
    const int x0 = xoff[b], nx = direct_xw(b, leafflag, range, n) ? xoff[b + 1] - x0 : 0;
    const int w0 = woff[b], nw = woff[b + 1] - w0;
    const uint64_t lt = lane_lt_mask();
    int at = mode ? noff[b] : 0, atf = mode ? wfoff[b] : 0;
    if (mode) {
        for (int k = lane; k < nu; k += 64) nidx[at + k] = uidx[u0 + k];
        for (int k = lane; k < nx; k += 64) nidx[at + nu + k] = xidx[x0 + k];
    }
    at += nu + nx;
    for (int k0 = 0; k0 < nw; k0 += 64) {
        const int k = k0 + lane;
        const int e = k < nw ? widx[w0 + k] : 0;
        const bool dir = k < nw && direct_xw(img_box(e), leafflag, range, n);
        const bool far = k < nw && !dir;
        const uint64_t md = __ballot(dir), mf = __ballot(far);
        if (mode) {
            if (dir) nidx[at + __popcll(md & lt)] = e;
            if (far) wfidx[atf + __popcll(mf & lt)] = e;
        }
        at += __popcll(md);
        atf += __popcll(mf);
    }
    if (!mode && lane == 0) {
        noff[b] = at;
        wfoff[b] = atf;
    }
}

// Leaves, and boxes that take P2L (an X list, and not summed point to point).
__global__ void k_flags(int B, const int* __restrict__ leafflag, const int2* __restrict__ range, int n,
                        const int* __restrict__ xcnt, int b2, int* __restrict__ fl, int* __restrict__ fx) {
    int b = blockIdx.x * TB + threadIdx.x;
    if (b == B) fl[B] = fx[B] = 0;   // the scans' last entries
    if (b >= B) return;
    fl[b] = leafflag[b];
    fx[b] = (b >= b2 && xcnt[b + 1] > xcnt[b] && !direct_xw(b, leafflag, range, n)) ? 1 : 0;
}

__global__ void k_zero3(int n, int* __restrict__ a, int* __restrict__ b, int* __restrict__ c) {
    const int i = blockIdx.x * TB + threadIdx.x;
    if (i < n) a[i] = b[i] = c[i] = 0;
}

__global__ void k_compact2(int B, const int* __restrict__ flag0, const int* __restrict__ off0, int* __restrict__ out0,
                           const int* __restrict__ flag1, const int* __restrict__ off1, int* __restrict__ out1) {
    int b = blockIdx.x * TB + threadIdx.x;
    if (b >= B) return;
    const int* flag = blockIdx.y ? flag1 : flag0;
    const int* off = blockIdx.y ? off1 : off0;
    int* out = blockIdx.y ? out1 : out0;
    if (flag[b]) out[off[b]] = b;
}

// Counts: V pairs, P2P point pairs (self pairs included), from the lists.
// V pairs: a grid-stride count over the dense table, one atomic per block.
__global__ void k_count_v(int64_t n, const int* __restrict__ vd, unsigned long long* __restrict__ out) {
    __shared__ unsigned long long part[TB / 64];
    unsigned long long c = 0;
    for (int64_t g = int64_t(blockIdx.x) * TB + threadIdx.x; g < n; g += int64_t(gridDim.x) * TB) c += vd[g] >= 0;
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < TB / 64; ++k) t += part[k];
        if (t) atomicAdd(&out[0], t);
    }
}

// Near-field point pairs of each leaf.
__global__ void k_counts(int B, const int* __restrict__ leafflag, const int2* __restrict__ range,
                         const int* __restrict__ uoff, const int* __restrict__ uidx,
                         unsigned long long* __restrict__ out) {
    int b = blockIdx.x * TB + threadIdx.x;
    unsigned long long pp = 0;
    if (b < B && leafflag[b]) {
        int2 r = range[b];
        unsigned long long nt = r.y - r.x;
        for (int k = uoff[b]; k < uoff[b + 1]; ++k) {
            int2 ra = range[img_box(uidx[k])];
            pp += nt * (unsigned long long)(ra.y - ra.x);
        }
    }
    if (pp) atomicAdd(&out[1], pp);
}

// Leaf work items of at most 64 targets, with cost estimates for ordering
// the near-field and leaf-evaluation launches heaviest first.
__global__ void k_item_count(int B, const int* __restrict__ nl_dev, const int* __restrict__ leaves,
                             const int2* __restrict__ range, int* __restrict__ cnt) {
    // entries nl .. B are zero, so that a scan of B + 1 entries ends with the total
    const int i = blockIdx.x * TB + threadIdx.x;
    if (i > B) return;
    if (i >= *nl_dev) {
        cnt[i] = 0;
        return;
    }
    const int2 r = range[leaves[i]];
    cnt[i] = (r.y - r.x + 63) / 64;
}

// One wave per leaf: the lanes sum the near-list source points, then take the
// leaf's items (up to 64 targets each) one per lane.
__global__ __launch_bounds__(256) void k_item_fill(int nl, const int* __restrict__ leaves,
                                                   const int2* __restrict__ range, const int* __restrict__ uoff,
                                                   const int* __restrict__ uidx, const int* __restrict__ woff, int b2,
                                                   const int* __restrict__ off, int2* __restrict__ items,
                                                   uint64_t* __restrict__ key_near, uint64_t* __restrict__ key_far,
                                                   uint32_t* __restrict__ id_near, uint32_t* __restrict__ id_far) {
    const int lane = threadIdx.x & 63, i = blockIdx.x * 4 + int(threadIdx.x >> 6);
    if (i >= nl) return;   // whole wave
    const int b = leaves[i];
    const int2 r = range[b];
    unsigned long long src = 0;
    for (int k = uoff[b] + lane; k < uoff[b + 1]; k += 64) {
        const int2 ra = range[img_box(uidx[k])];
        src += ra.y - ra.x;
    }
    for (int o = 32; o >= 1; o >>= 1) src += __shfl_xor(src, o, 64);
    const unsigned long long nfar = (b >= b2 ? 1 : 0) + (woff[b + 1] - woff[b]);
    const int nitem = (r.y - r.x + 63) / 64;
    for (int c = lane; c < nitem; c += 64) {
        const int at = off[i] + c, t0 = r.x + 64 * c;
        const unsigned long long nt = min(64, r.y - t0);
        items[at] = make_int2(b, t0);
        const unsigned long long cn = nt * src, cf = nt * nfar * 64;
        // heaviest first: 8-bit keys (one radix pass), descending in log2(cost)
        // in steps of 1/8 (costs within 9 % share a key and keep their order)
        key_near[at] = 0xffull - min(0xffull, (unsigned long long)(log2(double(cn) + 1.0) * 8.0));
        key_far[at] = 0xffull - min(0xffull, (unsigned long long)(log2(double(cf) + 1.0) * 8.0));
        id_near[at] = uint32_t(at);
        id_far[at] = uint32_t(at);
    }
}

__global__ void k_item_gather(int n, const int2* __restrict__ items, const uint32_t* __restrict__ idn,
                              const uint32_t* __restrict__ idf, int2* __restrict__ near, int2* __restrict__ far) {
    int i = blockIdx.x * TB + threadIdx.x;
    if (i >= n) return;
    near[i] = items[idn[i]];
    far[i] = items[idf[i]];
}

}  // namespace

// Host: the V-slot table, built once.
static const VTable& vtable_host() {
    static VTable t;
    static bool made = false;
    if (!made) {
        for (int o = 0; o < 8; ++o) {
            int ob[3] = {(o >> 2) & 1, (o >> 1) & 1, o & 1};
            // enumerate offsets in lexicographic order, pick those reachable from octant o
            int m = 0, j = 0;
            for (int dx = -3; dx <= 3; ++dx)
                for (int dy = -3; dy <= 3; ++dy)
                    for (int dz = -3; dz <= 3; ++dz) {
                        if (std::max(abs(dx), std::max(abs(dy), abs(dz))) <= 1) continue;
                        int d[3] = {dx, dy, dz};
                        bool ok = true;
                        int Dd[3], oc[3];
                        for (int k = 0; k < 3; ++k) {
                            int v = d[k] + ob[k];         // = 2 (D-1) + o'
                            int oo = ((v % 2) + 2) % 2;
                            int DD = (v - oo) / 2 + 1;
                            if (DD < 0 || DD > 2) ok = false;
                            Dd[k] = DD;
                            oc[k] = oo;
                        }
                        if (ok) {
                            t.D[o][j] = (unsigned char)(Dd[0] * 9 + Dd[1] * 3 + Dd[2]);
                            t.oc[o][j] = (unsigned char)((oc[0] << 2) | (oc[1] << 1) | oc[2]);
                            t.op[o][j] = short(m);
                            ++j;
                        }
                        ++m;
                    }
            if (j != kVPerOct) throw Error(KIFMM_ERR_STATE, "V table size");
        }
        made = true;
    }
    return t;
}

const void* vtable_host_ptr() { return &vtable_host(); }

void v_slot_offset(int o, int j, int d[3]) {
    const VTable& t = vtable_host();
    const int D = t.D[o][j], oc = t.oc[o][j];
    const int Dv[3] = {D / 9, (D / 3) % 3, D % 3};
    for (int k = 0; k < 3; ++k) d[k] = 2 * (Dv[k] - 1) + ((oc >> (2 - k)) & 1) - ((o >> (2 - k)) & 1);
}

// Read device ints through the plan's pinned words (one copy each, one wait).
struct IntPicks {
    const int* p[8];
    int n;
};

__global__ void k_pick_ints(IntPicks a, int* __restrict__ out) {
    if (int(threadIdx.x) < a.n) out[threadIdx.x] = *a.p[threadIdx.x];
}

// Read up to eight device ints: gathered into one staging word array by a
// one-wave kernel, then one copy and one synchronisation.
static void read_ints(kifmm_plan* P, hipStream_t s, std::initializer_list<const int*> src, int* dst) {
    int* h = reinterpret_cast<int*>(P->host.get());
    IntPicks a{};
    for (const int* d : src) {
        if (a.n == 8) throw Error(KIFMM_ERR_STATE, "too many values in one read-back");
        a.p[a.n++] = d;
    }
    if (a.n == 1) {
        KIFMM_HIP(hipMemcpyAsync(h, a.p[0], 4, hipMemcpyDeviceToHost, s));
    } else {
        P->readback.ensure(64);
        hipLaunchKernelGGL(k_pick_ints, dim3(1), dim3(64), 0, s, a, P->readback.as<int>());
        KIFMM_HIP(hipMemcpyAsync(h, P->readback.as<int>(), size_t(a.n) * 4, hipMemcpyDeviceToHost, s));
    }
    KIFMM_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < a.n; ++i) dst[i] = h[i];
}

static int read_int(kifmm_plan* P, const int* dptr, hipStream_t s) {
    int v = 0;
    read_ints(P, s, {dptr}, &v);
    return v;
}

// Re-sort from the order of the previous build (same N): keys in that order,
// the displaced subsequence D sorted and merged back into the rest R.  Writes
// the sorted keys and indices (P->keys, P->tmp_b) and returns true; returns
// false (nothing written that the full sort needs) when R is not in order or
// D is more than a quarter of the points (and more than one block sorts at
// once), for the caller's full sort.
static bool resort(kifmm_plan* P, double scale, hipStream_t s) {
    const int64_t N = P->N;
    const kifmm_options& o = P->opt;
    ++P->resort_steps;
    const size_t n1 = size_t(N) + 1;
    // flags, offsets, error word, D and R (keys and indices)
    const size_t need = n1 * 4 * 2 + 64 + size_t(N) * 12 * 2 + 256;
    P->resort.ensure(need);
    char* base = P->resort.as<char>();
    int* flag = reinterpret_cast<int*>(base);
    int* dpos = flag + n1;
    int* err = dpos + n1;
    uint64_t* dk = reinterpret_cast<uint64_t*>(base + ((n1 * 8 + 64 + 255) & ~size_t(255)));
    uint64_t* rk = dk + N;
    uint32_t* dv = reinterpret_cast<uint32_t*>(rk + N);
    uint32_t* rv = dv + N;
    uint64_t* ka = P->tmp_c.as<uint64_t>();
    uint32_t* va = P->tmp_d.as<uint32_t>();
    int* bad = P->flag.as<int>();
    hipLaunchKernelGGL(k_keys_prev, dim3(nblocks(N)), dim3(TB), 0, s, P->x64.as<double>(), N, P->lo[0], P->lo[1],
                       P->lo[2], scale, P->side, o.explicit_root, P->perm.as<int>(), ka, va, bad);
    hipLaunchKernelGGL(k_displaced, dim3(nblocks(N + 1)), dim3(TB), 0, s, ka, va, N, flag, err);
    exclusive_scan<int>(P, flag, dpos, N + 1, s);
    hipLaunchKernelGGL(k_split_dr, dim3(nblocks(N)), dim3(TB), 0, s, ka, va, N, flag, dpos, dk, dv, rk, rv);
    hipLaunchKernelGGL(k_check_sorted, dim3(nblocks(N)), dim3(TB), 0, s, rk, rv, N, dpos, err);
    int h[2];
    read_ints(P, s, {dpos + N, err}, h);
    const int64_t nd = h[0], nr = N - nd;
    if (h[1] || (nd > N / 4 && nd > RS_TILE)) return false;
    if (nd > 0) {
        // D by key (stable, so equal keys stay in their previous order), then
        // equal keys by index; the scratch of the full sort is free here
        radix_sort(P, dk, dv, ka, va, nd, 63, s);
        hipLaunchKernelGGL(k_fix_ties, dim3(nblocks(nd)), dim3(TB), 0, s, dk, dv, nd);
    }
    uint64_t* keys = P->keys.as<uint64_t>();
    uint32_t* idx = P->tmp_b.as<uint32_t>();
    if (nr > 0)
        hipLaunchKernelGGL(k_merge_into, dim3(nblocks(nr)), dim3(TB), 0, s, rk, rv, nr, dk, dv, nd, keys, idx);
    if (nd > 0)
        hipLaunchKernelGGL(k_merge_into, dim3(nblocks(nd)), dim3(TB), 0, s, dk, dv, nd, rk, rv, nr, keys, idx);
    ++P->resort_hits;
    return true;
}

void build_tree(kifmm_plan* P, const double* positions, hipStream_t s) {
    const int64_t N = P->N;
    const kifmm_options& o = P->opt;
    // positions copy
    P->x64.ensure(size_t(N) * 24);
    KIFMM_HIP(hipMemcpyAsync(P->x64.p, positions, size_t(N) * 24, hipMemcpyDeviceToDevice, s));
    P->flag.ensure(64);
    int* bad = P->flag.as<int>();
    KIFMM_HIP(hipMemsetAsync(bad, 0, 64, s));

    // root cube
    if (o.explicit_root) {
        for (int d = 0; d < 3; ++d) P->lo[d] = o.root_lo[d];
        P->side = o.root_side;
    } else {
        int nb = std::min<int64_t>(1024, (N + TB - 1) / TB);
        P->tmp_a.ensure(size_t(nb) * 6 * 8);
        hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(TB), 0, s, P->x64.as<double>(), N, P->tmp_a.as<double>(), bad);
        std::vector<double> part(size_t(nb) * 6);
        int hbad = 0;
        KIFMM_HIP(hipMemcpyAsync(part.data(), P->tmp_a.p, part.size() * 8, hipMemcpyDeviceToHost, s));
        KIFMM_HIP(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s));
        KIFMM_HIP(hipStreamSynchronize(s));
        if (hbad) throw Error(KIFMM_ERR_INPUT, "non-finite position");
        double mn[3] = {1e308, 1e308, 1e308}, mx[3] = {-1e308, -1e308, -1e308};
        for (int b = 0; b < nb; ++b)
            for (int d = 0; d < 3; ++d) {
                mn[d] = std::min(mn[d], part[6 * b + d]);
                mx[d] = std::max(mx[d], part[6 * b + 3 + d]);
            }
        double ext = std::max(mx[0] - mn[0], std::max(mx[1] - mn[1], mx[2] - mn[2]));
        double sd = 1.0;
        if (ext > 0) {
            int e = 0;
            double m = frexp(ext * (1.0 + ldexp(1.0, -10)), &e);
            sd = (m == 0.5) ? ldexp(1.0, e - 1) : ldexp(1.0, e);
        }
        P->side = sd;
        for (int d = 0; d < 3; ++d) P->lo[d] = floor(mn[d] * 4096.0 / sd) * sd / 4096.0;
    }

    // keys and sort
    P->keys.ensure(size_t(N) * 8);
    P->tmp_b.ensure(size_t(N) * 4);   // idx
    P->tmp_c.ensure(size_t(N) * 8);   // key tmp
    P->tmp_d.ensure(size_t(N) * 4);   // idx tmp
    uint64_t* keys = P->keys.as<uint64_t>();
    uint32_t* idx = P->tmp_b.as<uint32_t>();
    double scale = ldexp(1.0, kBits) / P->side;
    // a flagged point gets key 0, so the build below stays in bounds; the flag
    // is read with the final counts
    const bool prev_order = P->sorted_valid;
    P->sorted_valid = false;
    ++P->builds;
    if (!(prev_order && resort(P, scale, s))) {
        hipLaunchKernelGGL(k_keys, dim3(nblocks(N)), dim3(TB), 0, s, P->x64.as<double>(), N, P->lo[0], P->lo[1],
                           P->lo[2], scale, P->side, o.explicit_root, keys, idx, bad);
        radix_sort(P, keys, idx, P->tmp_c.as<uint64_t>(), P->tmp_d.as<uint32_t>(), N, 63, s);
    }
    P->xs.ensure(size_t(N) * 16);
    P->perm.ensure(size_t(N) * 4);
    hipLaunchKernelGGL(k_gather_pos, dim3(nblocks(N)), dim3(TB), 0, s, P->x64.as<double>(), idx, N,
                       P->xs.as<float4>(), P->perm.as<int>());

    // levels
    int Lu = 0;
    while (Lu < o.max_depth && double(P->leaf) * pow(8.0, Lu) < double(N)) ++Lu;
    int64_t cap = std::max<int64_t>(1024, 4 * (N / std::max(1, P->leaf)) + 64);
    auto ensure_boxes = [&](int64_t need, int64_t keep) {
        P->bx_anchor.grow(size_t(need) * 16, size_t(keep) * 16, s);
        P->bx_range.grow(size_t(need) * 8, size_t(keep) * 8, s);
        P->bx_parent.grow(size_t(need) * 4, size_t(keep) * 4, s);
        P->bx_child.grow(size_t(need) * 8, size_t(keep) * 8, s);
        P->bx_leaf.grow(size_t(need) * 4, size_t(keep) * 4, s);
        P->bx_mkey.grow(size_t(need) * 8, size_t(keep) * 8, s);
        P->nonleaf.grow(size_t(need) * 4, size_t(keep) * 4, s);
    };
    ensure_boxes(cap, 0);
    int root_leaf = o.adaptive ? (N <= P->leaf || o.max_depth == 0) : (Lu == 0);
    // a small tree builds every level in one block, which writes the root too
    const bool small_tree = N <= kSmallTreeN && !root_leaf;
    if (!small_tree)
        hipLaunchKernelGGL(k_root, dim3(1), dim3(1), 0, s, int(N), root_leaf, P->bx_anchor.as<int4>(),
                           P->bx_range.as<int2>(), P->bx_parent.as<int>(), P->bx_child.as<int2>(),
                           P->bx_leaf.as<int>(), P->bx_mkey.as<uint64_t>(), P->nonleaf.as<int>());
    P->lev.clear();
    LevelInfo L0;
    L0.start = 0;
    L0.count = 1;
    L0.nl_start = 0;
    L0.nl_count = root_leaf ? 0 : 1;
    P->lev.push_back(L0);
    int64_t total = 1, nl_total = L0.nl_count;
    // a small tree: every level in one block, one read-back of the level table
    bool levels_done = false;
    if (small_tree) {
        const int ncap = int(cap);
        P->tmp_a.ensure(size_t(ncap) * 9 * 4 + size_t(ncap + 1) * 16 + size_t(kMaxLevels + 1) * 16 + 256);
        char* base = P->tmp_a.as<char>();
        int* bounds = reinterpret_cast<int*>(base);
        unsigned long long* cnt = reinterpret_cast<unsigned long long*>(base + ((size_t(ncap) * 9 * 4 + 15) & ~size_t(15)));
        unsigned long long* offs = cnt + (ncap + 1);
        int4* levt = reinterpret_cast<int4*>(offs + (ncap + 1));
        int* levn = reinterpret_cast<int*>(levt + (kMaxLevels + 1));
        hipLaunchKernelGGL(k_levels_block, dim3(1), dim3(LB_THREADS), 0, s, keys, ncap, ncap, bounds, cnt, offs,
                           P->bx_anchor.as<int4>(), P->bx_range.as<int2>(), P->bx_parent.as<int>(),
                           P->bx_child.as<int2>(), P->bx_leaf.as<int>(), P->bx_mkey.as<uint64_t>(),
                           P->nonleaf.as<int>(), levt, levn, P->leaf, o.adaptive, o.max_depth, Lu, 1, int(N));
        // the level table and, right after it, the two counters in one copy
        static_assert((kMaxLevels + 1) * 16 + 8 <= 512, "host words");
        int* hw = reinterpret_cast<int*>(P->host.get());
        KIFMM_HIP(hipMemcpyAsync(hw, levt, size_t(kMaxLevels + 1) * 16 + 8, hipMemcpyDeviceToHost, s));
        KIFMM_HIP(hipStreamSynchronize(s));
        const int* hn = hw + 4 * (kMaxLevels + 1);
        if (hn[1] == 0) {
            const int nlev = hn[0];
            P->lev.clear();
            for (int l = 0; l < nlev; ++l) {
                LevelInfo li;
                li.start = hw[4 * l];
                li.count = hw[1 + 4 * l];
                li.nl_start = hw[2 + 4 * l];
                li.nl_count = hw[3 + 4 * l];
                P->lev.push_back(li);
            }
            total = P->lev.back().start + P->lev.back().count;
            levels_done = true;
        }
        // else: storage or scratch would overflow; build the levels below
    }
    for (int l = 0; !levels_done; ++l) {
        const LevelInfo cur = P->lev[l];
        if (cur.nl_count == 0) break;
        int nf = int(cur.nl_count);
        const size_t bwords = (size_t(nf) * 9 + 1) & ~size_t(1);   // 8-byte aligned after the bounds
        P->tmp_a.ensure(bwords * 4 + size_t(nf + 1) * 8 + 64);
        int* bounds = P->tmp_a.as<int>();
        unsigned long long* cnt = reinterpret_cast<unsigned long long*>(bounds + bwords);
        // tmp_e holds the scan (nf+1 packed offsets)
        P->tmp_e.ensure(size_t(nf + 1) * 8 + 64);
        unsigned long long* off = P->tmp_e.as<unsigned long long>();
        const int* front = P->nonleaf.as<int>() + cur.nl_start;
        hipLaunchKernelGGL(k_split, dim3(nblocks(int64_t(nf) * 64)), dim3(TB), 0, s, front, nf, l, keys,
                           P->bx_range.as<int2>(), bounds, cnt, P->leaf, o.adaptive, o.max_depth, Lu);
        exclusive_scan<unsigned long long>(P, cnt, off, nf + 1, s);
        unsigned long long* hw = P->host.get();
        KIFMM_HIP(hipMemcpyAsync(hw, off + nf, 8, hipMemcpyDeviceToHost, s));
        KIFMM_HIP(hipStreamSynchronize(s));
        LevelInfo nx;
        nx.start = total;
        nx.count = int64_t(hw[0] & 0xffffffffull);
        nx.nl_start = nl_total;
        nx.nl_count = int64_t(hw[0] >> 32);
        if (total + nx.count > cap) {
            int64_t ncap = std::max<int64_t>(2 * cap, total + nx.count + 64);
            ensure_boxes(ncap, total);
            cap = ncap;
            front = P->nonleaf.as<int>() + cur.nl_start;
        }
        hipLaunchKernelGGL(k_emit, dim3(nblocks(int64_t(nf) * 8)), dim3(TB), 0, s, front, nf, l, keys, bounds, off,
                           int(nx.start), int(nx.nl_start), P->bx_anchor.as<int4>(), P->bx_range.as<int2>(),
                           P->bx_parent.as<int>(), P->bx_child.as<int2>(), P->bx_leaf.as<int>(),
                           P->bx_mkey.as<uint64_t>(), P->nonleaf.as<int>(), P->leaf, o.adaptive, o.max_depth, Lu);
        total += nx.count;
        nl_total += nx.nl_count;
        P->lev.push_back(nx);
        if (int(P->lev.size()) > kMaxLevels) throw Error(KIFMM_ERR_STATE, "tree deeper than the key resolution");
    }
    P->B = total;
    P->depth = int(P->lev.size()) - 1;
    const int B = int(total);
    if (P->periodic && B > kBoxMask) throw Error(KIFMM_ERR_INPUT, "too many boxes for periodic list entries");
    // first box with a downward density: level 2 in free space, the root when periodic
    const int b2 = P->periodic ? 0 : (P->depth >= 2 ? int(P->lev[2].start) : B);
    P->bfar = b2;

    LevelTable lt{};
    for (int l = 0; l <= P->depth; ++l) {
        lt.start[l] = int(P->lev[l].start);
        lt.count[l] = int(P->lev[l].count);
    }
    // colleagues
    P->coll.ensure(size_t(B) * 27 * 4);
    hipLaunchKernelGGL(k_colleagues, dim3(nblocks(int64_t(B) * 27)), dim3(TB), 0, s, B, P->bx_anchor.as<int4>(),
                       P->bx_mkey.as<uint64_t>(), lt, P->periodic ? 1 : 0, P->coll.as<int>());
    // V dense table
    static DBuf* vt_dev = nullptr;   // per process, small
    if (!vt_dev) {
        vt_dev = new DBuf();
        vt_dev->ensure(sizeof(VTable));
        KIFMM_HIP(hipMemcpy(vt_dev->p, &vtable_host(), sizeof(VTable), hipMemcpyHostToDevice));
    }
    int nvb = B - b2;
    P->vdense.ensure(size_t(std::max(nvb, 1)) * kVPerOct * 4);
    if (nvb > 0)
        hipLaunchKernelGGL(k_vdense, dim3(nblocks(int64_t(nvb) * 64)), dim3(TB), 0, s, b2, nvb, P->bx_anchor.as<int4>(),
                           P->bx_parent.as<int>(), P->bx_child.as<int2>(), P->bx_leaf.as<int>(), P->coll.as<int>(),
                           vt_dev->as<VTable>(), P->vdense.as<int>());
    // coarse adjacent leaves, top-down
    P->cal.ensure(size_t(B) * 26 * 4);   // every row below the root is written by k_cal
    for (int l = 1; l <= P->depth; ++l)
        hipLaunchKernelGGL(k_cal, dim3(nblocks(P->lev[l].count, 4)), dim3(TB), 0, s, int(P->lev[l].start),
                           int(P->lev[l].count), P->bx_anchor.as<int4>(), P->bx_parent.as<int>(),
                           P->bx_leaf.as<int>(), P->coll.as<int>(), P->cal.as<int>(), bad);
    // X lists (rows over all boxes; non-empty from the first far-field level)
    P->x_off.ensure(size_t(B + 1) * 4);
    int* xoff = P->x_off.as<int>();
    P->u_off.ensure(size_t(B + 1) * 4);
    int* uoff = P->u_off.as<int>();
    P->tmp_e.ensure(size_t(B + 1) * 4);
    int* cursor = P->tmp_e.as<int>();
    P->w_off.ensure(size_t(B + 1) * 4);
    int* woff = P->w_off.as<int>();
    // the X, U and W counts start at zero: one launch for the three
    hipLaunchKernelGGL(k_zero3, dim3(nblocks(B + 1)), dim3(TB), 0, s, B + 1, xoff, uoff, woff);
    // List storage is sized by bounds, so that no size is read back here:
    // X(b) <= 26 leaf colleagues of the parent + 26 coarse adjacent leaves of
    // the parent; U(b) <= 27 + 26 of its own, and the finer part adds one
    // entry per coarse-adjacent entry of a finer leaf (<= 26 per box); W is X
    // transposed.  The sizes themselves are read with the final counts.
    const size_t xcap = size_t(std::max(nvb, 1)) * 52, ucap = size_t(B) * (53 + 26);
    P->x_idx.ensure(xcap * 4);
    P->u_idx.ensure(ucap * 4);
    P->w_idx.ensure(xcap * 4);
    ListArgs la{b2, nvb, B, P->bx_anchor.as<int4>(), P->bx_parent.as<int>(), P->bx_leaf.as<int>(), P->coll.as<int>(),
                P->cal.as<int>(), xoff, P->x_idx.as<int>(), uoff, P->u_idx.as<int>(), woff, P->w_idx.as<int>(),
                cursor};
    const int nbx = nvb > 0 ? nblocks(nvb, 4) : 0, nbu = nblocks(B, 4);
    // counts of X, of the own and the finer part of U (one launch), their scans
    // (one launch when small), the X entries with the own part of U, then the
    // finer part of U with the W counts (which read the X entries)
    hipLaunchKernelGGL(k_list_counts, dim3(nbx + 2 * nbu), dim3(TB), 0, s, la, nbx, nbu);
    exclusive_scan2<int>(P, xoff, xoff, nullptr, B + 1, uoff, uoff, B + 1, s);
    hipLaunchKernelGGL(k_list_fill_a, dim3(nbx + nbu), dim3(TB), 0, s, la, nbx);
    hipLaunchKernelGGL(k_list_fill_b, dim3(nbu + nbx), dim3(TB), 0, s, la, nbu);
    // W = X transposed: the scan also leaves the cursor (a copy of the offsets)
    exclusive_scan2<int>(P, woff, woff, cursor, B + 1, nullptr, nullptr, 0, s);
    if (nvb > 0) hipLaunchKernelGGL(k_list_fill_w, dim3(nbx), dim3(TB), 0, s, la);
    // every row of X, U and W ascending (U and W were filled through atomics)
    hipLaunchKernelGGL(k_sort_rows, dim3(B, 3), dim3(64), 0, s, B, xoff, P->x_idx.as<int>(), uoff,
                       P->u_idx.as<int>(), woff, P->w_idx.as<int>());
    // near lists (U plus the W/X pairs summed point to point) and the W lists
    // of the leaf evaluation (the other W pairs)
    P->n_off.ensure(size_t(B + 1) * 4);
    P->wf_off.ensure(size_t(B + 1) * 4);
    int* noff = P->n_off.as<int>();
    int* wfoff = P->wf_off.as<int>();
    hipLaunchKernelGGL(k_near, dim3(nblocks(B + 1, 4)), dim3(TB), 0, s, B, P->n, P->bx_leaf.as<int>(),
                       P->bx_range.as<int2>(), uoff, P->u_idx.as<int>(), xoff, P->x_idx.as<int>(), woff,
                       P->w_idx.as<int>(), noff, (int*)nullptr, wfoff, (int*)nullptr, 0);
    exclusive_scan2<int>(P, noff, noff, nullptr, B + 1, wfoff, wfoff, B + 1, s);
    P->n_idx.ensure((ucap + 2 * xcap) * 4);
    P->wf_idx.ensure(xcap * 4);
    hipLaunchKernelGGL(k_near, dim3(nblocks(B + 1, 4)), dim3(TB), 0, s, B, P->n, P->bx_leaf.as<int>(),
                       P->bx_range.as<int2>(), uoff, P->u_idx.as<int>(), xoff, P->x_idx.as<int>(), woff,
                       P->w_idx.as<int>(), noff, P->n_idx.as<int>(), wfoff, P->wf_idx.as<int>(), 1);
    // leaf list and X-box list
    P->tmp_f.ensure(size_t(B + 1) * 4 * 3);
    int* fl = P->tmp_f.as<int>();
    int* ol = fl + (B + 1);
    int* ox = ol + (B + 1);
    // the X-box flags are kept: a box's downward check potential is written by
    // the P2L kernel exactly when its flag is set
    P->xflag.ensure(size_t(B + 1) * 4);
    int* fx = P->xflag.as<int>();
    hipLaunchKernelGGL(k_flags, dim3(nblocks(B + 1)), dim3(TB), 0, s, B, P->bx_leaf.as<int>(), P->bx_range.as<int2>(),
                       P->n, xoff, b2, fl, fx);
    exclusive_scan2<int>(P, fl, ol, nullptr, B + 1, fx, ox, B + 1, s);
    // the leaf and X-box lists are sized by B, so that every size of the build
    // is read back once, below
    P->leaves.ensure(size_t(B) * 4);
    P->xboxes.ensure(size_t(B) * 4);
    if (B > 0)
        hipLaunchKernelGGL(k_compact2, dim3(nblocks(B), 2), dim3(TB), 0, s, B, fl, ol, P->leaves.as<int>(), fx, ox,
                           P->xboxes.as<int>());
    // work items per leaf (at most 64 targets each)
    P->tmp_a.ensure(size_t(B + 1) * 8 + 64);
    int* icnt = P->tmp_a.as<int>();
    int* ioff = icnt + (B + 1);
    hipLaunchKernelGGL(k_item_count, dim3(nblocks(B + 1)), dim3(TB), 0, s, B, ol + B, P->leaves.as<int>(),
                       P->bx_range.as<int2>(), icnt);
    exclusive_scan<int>(P, icnt, ioff, B + 1, s);
    // sizes: leaves, X boxes, items, the input flags, list lengths X, U, W
    int hs[7];
    read_ints(P, s, {ol + B, ox + B, ioff + B, bad, xoff + B, uoff + B, woff + B}, hs);
    const int nl = hs[0], nxb = hs[1], ni = hs[2], hbad = hs[3], nx = hs[4], nu = hs[5], nw = hs[6];
    if (hbad & 1)
        throw Error(KIFMM_ERR_INPUT, o.explicit_root ? "non-finite position or point outside the explicit root"
                                                     : "non-finite position");
    if (hbad & 2) throw Error(KIFMM_ERR_STATE, "more than 26 coarse adjacent leaves");
    P->nleaves = nl;
    P->n_xboxes = nxb;
    P->n_items = ni;
    // leaf work items, heaviest first
    {
        P->item_tmp.ensure(size_t(ni) * (8 + 8 + 8 + 4 + 4 + 4 + 4) + 1024);
        char* base = P->item_tmp.as<char>();
        int2* items = reinterpret_cast<int2*>(base);
        uint64_t* kn = reinterpret_cast<uint64_t*>(base + size_t(ni) * 8);
        uint64_t* kf = kn + ni;
        uint32_t* idn = reinterpret_cast<uint32_t*>(kf + ni);
        uint32_t* idf = idn + ni;
        uint32_t* vtmp = idf + ni;
        P->tmp_c.ensure(size_t(ni) * 8);
        hipLaunchKernelGGL(k_item_fill, dim3(nblocks(nl, 4)), dim3(TB), 0, s, nl, P->leaves.as<int>(),
                           P->bx_range.as<int2>(), noff, P->n_idx.as<int>(), wfoff, b2, ioff, items, kn, kf, idn, idf);
        // a grid this small runs in one round on the chip, where the order
        // of the items does not matter: leaf order (the identity ids)
        if (ni > kItemOrderMin) {
            radix_sort(P, kn, idn, P->tmp_c.as<uint64_t>(), vtmp, ni, 8, s);
            radix_sort(P, kf, idf, P->tmp_c.as<uint64_t>(), vtmp, ni, 8, s);
        }
        P->items_near.ensure(size_t(ni) * 8);
        P->items_far.ensure(size_t(ni) * 8);
        hipLaunchKernelGGL(k_item_gather, dim3(nblocks(ni)), dim3(TB), 0, s, ni, items, idn, idf,
                           P->items_near.as<int2>(), P->items_far.as<int2>());
    }
    // counts (the pair counts are taken on request: count_pairs)
    P->counts[0] = B;
    P->counts[1] = nl;
    P->counts[2] = P->depth;
    P->counts[3] = 0;
    P->counts[4] = 0;
    P->pairs_counted = false;
    P->counts[5] = nw;
    P->counts[6] = nx;
    P->counts[7] = nu;
    P->counts[8] = N;
    P->counts[9] = P->n;
    P->sorted_valid = true;   // perm is this build's order: the next build may start from it
}

void count_pairs(kifmm_plan* P, hipStream_t s) {
    const int B = int(P->B), nvb = B - int(P->bfar);
    P->pair_cnt.ensure(64);
    unsigned long long* dc = P->pair_cnt.as<unsigned long long>();
    KIFMM_HIP(hipMemsetAsync(dc, 0, 16, s));
    if (nvb > 0)
        hipLaunchKernelGGL(k_count_v, dim3(std::min(1024, nblocks(int64_t(nvb) * kVPerOct))), dim3(TB), 0, s,
                           int64_t(nvb) * kVPerOct, P->vdense.as<int>(), dc);
    if (B > 0)
        hipLaunchKernelGGL(k_counts, dim3(nblocks(B)), dim3(TB), 0, s, B, P->bx_leaf.as<int>(),
                           P->bx_range.as<int2>(), P->n_off.as<int>(), P->n_idx.as<int>(), dc);
    unsigned long long* hw = P->host.get();
    KIFMM_HIP(hipMemcpyAsync(hw, dc, 16, hipMemcpyDeviceToHost, s));
    KIFMM_HIP(hipStreamSynchronize(s));
    P->counts[3] = int64_t(hw[0]);
    P->counts[4] = int64_t(hw[1]);
    P->pairs_counted = true;
}

}  // namespace kifmm
