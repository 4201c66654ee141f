// Clump aggregation (Section 2.4): the long-range forces act on the pebbles
// and are summed, with their moments, into the force and torque of each clump.
//
// Segmented reduction over the pebbles in caller order.  A block takes 256
// consecutive pebbles; each thread forms its pebble's terms in FP64 and the
// block runs a segmented scan keyed by clump (a fixed tree order), so every
// clump that lies inside one block is finished there.  A clump that crosses a
// block boundary is finished by a second kernel, one thread per clump, which
// adds the boundary segments of the blocks it covers in block order from a
// small partial buffer (two segments of NV doubles per block).  Both orders
// are fixed, so the result is deterministic; it equals the caller-order sum
// up to FP64 rounding.
//
// The clump of a pebble comes from the clump ids registered with the plan, or
// from a binary search of the CSR offsets of the call.  Offsets are checked on
// the device: a clump whose range is not a valid CSR row (or offsets[0] != 0)
// gets NaN results and sets the plan's input-error word, which the next
// kifmm_synchronize reports; reads stay inside the buffers in every case.
#include <math.h>

#include <mutex>

#include "common.h"

namespace kifmm {

namespace {

constexpr int CB = 256;   // pebbles per block

// Clump of pebble k (caller order), or -1 for none.
__device__ inline int64_t clump_of(int64_t k, const int* __restrict__ cid, const int64_t* __restrict__ off,
                                   int64_t C) {
    if (cid) return cid[k];
    // largest c in [0, C) with off[c] <= k, kept only when k < off[c + 1]
    int64_t lo = 0, hi = C;   // invariant: off[c] <= k for c < lo (once lo > 0)
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= k) lo = mid + 1;
        else hi = mid;
    }
    const int64_t c = lo - 1;
    if (c < 0 || k >= off[c + 1]) return -1;
    return c;
}

// Segmented inclusive scan of NV doubles over the block, keyed by clump;
// afterwards v holds the sum of this thread's segment up to and including it.
template <int NV>
__device__ inline void seg_scan(double (&v)[NV], int64_t key, double (*s)[CB], int64_t* keys) {
    const int t = threadIdx.x;
    keys[t] = key;
#pragma unroll
    for (int q = 0; q < NV; ++q) s[q][t] = v[q];
    __syncthreads();
    for (int d = 1; d < CB; d <<= 1) {
        const bool take = t >= d && keys[t - d] == key;
        double a[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) a[q] = take ? s[q][t - d] : 0.0;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            v[q] += a[q];
            s[q][t] = v[q];
        }
        __syncthreads();
    }
}

// Clump total q (of NV) to the outputs: q < 3 to oa[c][3], q >= 3 to ob[c][3].
__device__ inline void put(double* __restrict__ oa, double* __restrict__ ob, int64_t c, int q, double v) {
    if (q < 3) oa[size_t(c) * 3 + q] = v;
    else ob[size_t(c) * 3 + q - 3] = v;
}

// After seg_scan: write the totals of clumps inside this block to the outputs
// and the block's first and last segments to part[blk][2][NV].
template <int NV>
__device__ inline void seg_finish(const double (&v)[NV], int64_t key, const int64_t* keys, int64_t b0, int64_t C,
                                  const int64_t* __restrict__ off, double* __restrict__ oa, double* __restrict__ ob,
                                  double* __restrict__ part) {
    const int t = threadIdx.x;
    const bool tail = t == CB - 1 || keys[t + 1] != key;
    if (!tail) return;
    if (keys[0] == key) {   // the segment holding thread 0
#pragma unroll
        for (int q = 0; q < NV; ++q) part[(size_t(blockIdx.x) * 2) * NV + q] = v[q];
    }
    if (t == CB - 1) {
#pragma unroll
        for (int q = 0; q < NV; ++q) part[(size_t(blockIdx.x) * 2 + 1) * NV + q] = v[q];
    }
    if (key < 0 || key >= C) return;
    const int64_t a = off[key], b = off[key + 1];
    if (a >= b0 && b <= b0 + CB && a < b) {
#pragma unroll
        for (int q = 0; q < NV; ++q) put(oa, ob, key, q, v[q]);
    }
}

// Clumps that cross a block boundary (and empty ones, and the offset checks):
// one thread per clump.  With null outputs only the checks run.
template <int NV>
__global__ void k_clump_fix(int64_t C, int64_t N, const int64_t* __restrict__ off, const double* __restrict__ part,
                            double* __restrict__ oa, double* __restrict__ ob, int* __restrict__ err, int check) {
    const int64_t c = blockIdx.x * int64_t(CB) + threadIdx.x;
    if (c >= C) return;
    const int64_t a = off[c], b = off[c + 1];
    if (check && (a > b || a < 0 || b > N || (c == 0 && a != 0))) {
        atomicOr(err, 1);
        if (oa)
#pragma unroll
            for (int q = 0; q < NV; ++q) put(oa, ob, c, q, NAN);
        return;
    }
    if (!oa) return;
    if (a == b) {
#pragma unroll
        for (int q = 0; q < NV; ++q) put(oa, ob, c, q, 0.0);
        return;
    }
    const int64_t bl0 = a / CB, bl1 = (b - 1) / CB;
    if (bl0 == bl1) return;   // finished by its block
    double s[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) s[q] = part[(size_t(bl0) * 2 + 1) * NV + q];
    for (int64_t bl = bl0 + 1; bl < bl1; ++bl)
#pragma unroll
        for (int q = 0; q < NV; ++q) s[q] += part[(size_t(bl) * 2) * NV + q];
#pragma unroll
    for (int q = 0; q < NV; ++q) put(oa, ob, c, q, s[q] + part[(size_t(bl1) * 2) * NV + q]);
}

// Per-pebble force q_k E_k and moment (x_k - X_c) x q_k E_k, reduced per clump
// into F[c] and T[c].
__global__ __launch_bounds__(CB) void k_clump(int64_t N, int64_t C, const int64_t* __restrict__ off,
                                              const int* __restrict__ cid, const double* __restrict__ x,
                                              const float* __restrict__ q, const float* __restrict__ E,
                                              const double* __restrict__ cen, double* __restrict__ F,
                                              double* __restrict__ T, double* __restrict__ part) {
    __shared__ double s[6][CB];
    __shared__ int64_t keys[CB];
    const int64_t b0 = blockIdx.x * int64_t(CB);
    const int64_t k = b0 + threadIdx.x;
    const int64_t c = k < N ? clump_of(k, cid, off, C) : -1;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (c >= 0) {
        const double qk = q[k];
        const double gx = qk * double(E[3 * k]), gy = qk * double(E[3 * k + 1]), gz = qk * double(E[3 * k + 2]);
        const double rx = x[3 * k] - cen[3 * c], ry = x[3 * k + 1] - cen[3 * c + 1], rz = x[3 * k + 2] - cen[3 * c + 2];
        v[0] = gx;
        v[1] = gy;
        v[2] = gz;
        v[3] = ry * gz - rz * gy;
        v[4] = rz * gx - rx * gz;
        v[5] = rx * gy - ry * gx;
    }
    seg_scan<6>(v, c, s, keys);
    seg_finish<6>(v, c, keys, b0, C, off, F, T, part);
}

// Backward of the aggregation for dL/dF_c = Fb, dL/dT_c = Tb (either may be
// null = 0), with r_k = x_k - X_c:
//   dL/dq_k = Fb.E_k + Tb.(r_k x E_k),  dL/dE_k = q_k (Fb + Tb x r_k),
//   dL/dx_k = q_k (E_k x Tb),           dL/dX_c = -sum_k dL/dx_k.
// Pebbles outside every clump get zeros.  `acc`: dL/dq and dL/dx are added to
// qb and xb instead of stored.  The clump sum of -dL/dx_k goes to Xb.
__global__ __launch_bounds__(CB) void k_clump_bwd(int64_t N, int64_t C, const int64_t* __restrict__ off,
                                                  const int* __restrict__ cid, const double* __restrict__ x,
                                                  const float* __restrict__ q, const float* __restrict__ E,
                                                  const double* __restrict__ cen, const double* __restrict__ Fb,
                                                  const double* __restrict__ Tb, float* __restrict__ qb,
                                                  float* __restrict__ Eb, float* __restrict__ xb, int acc,
                                                  double* __restrict__ Xb, double* __restrict__ part) {
    __shared__ double s[3][CB];
    __shared__ int64_t keys[CB];
    const int64_t b0 = blockIdx.x * int64_t(CB);
    const int64_t k = b0 + threadIdx.x;
    const int64_t c = k < N ? clump_of(k, cid, off, C) : -1;
    double g[3] = {0, 0, 0}, m[3] = {0, 0, 0};
    if (c >= 0) {
        const double f0 = Fb ? Fb[3 * c] : 0.0, f1 = Fb ? Fb[3 * c + 1] : 0.0, f2 = Fb ? Fb[3 * c + 2] : 0.0;
        const double t0 = Tb ? Tb[3 * c] : 0.0, t1 = Tb ? Tb[3 * c + 1] : 0.0, t2 = Tb ? Tb[3 * c + 2] : 0.0;
        const double qk = q[k];
        const double e0 = E[3 * k], e1 = E[3 * k + 1], e2 = E[3 * k + 2];
        const double r0 = x[3 * k] - cen[3 * c], r1 = x[3 * k + 1] - cen[3 * c + 1], r2 = x[3 * k + 2] - cen[3 * c + 2];
        // r x E, Tb x r, q E x Tb
        const double c0 = r1 * e2 - r2 * e1, c1 = r2 * e0 - r0 * e2, c2 = r0 * e1 - r1 * e0;
        const double d0 = t1 * r2 - t2 * r1, d1 = t2 * r0 - t0 * r2, d2 = t0 * r1 - t1 * r0;
        g[0] = qk * (e1 * t2 - e2 * t1);
        g[1] = qk * (e2 * t0 - e0 * t2);
        g[2] = qk * (e0 * t1 - e1 * t0);
        const float gq = float((f0 * e0 + f1 * e1 + f2 * e2) + (t0 * c0 + t1 * c1 + t2 * c2));
        if (qb) qb[k] = acc ? qb[k] + gq : gq;
        if (Eb) {
            Eb[3 * k] = float(qk * (f0 + d0));
            Eb[3 * k + 1] = float(qk * (f1 + d1));
            Eb[3 * k + 2] = float(qk * (f2 + d2));
        }
        if (xb)
            for (int d = 0; d < 3; ++d) xb[3 * k + d] = acc ? xb[3 * k + d] + float(g[d]) : float(g[d]);
        for (int d = 0; d < 3; ++d) m[d] = -g[d];
    } else if (k < N && !acc) {
        if (qb) qb[k] = 0.f;
        for (int d = 0; d < 3; ++d) {
            if (Eb) Eb[3 * k + d] = 0.f;
            if (xb) xb[3 * k + d] = 0.f;
        }
    } else if (k < N && Eb) {
        for (int d = 0; d < 3; ++d) Eb[3 * k + d] = 0.f;
    }
    if (!Xb) return;   // block-uniform
    seg_scan<3>(m, c, s, keys);
    seg_finish<3>(m, c, keys, b0, C, off, Xb, nullptr, part);
}

// caller-order clump ids from CSR offsets (checked on the host)
__global__ void k_clump_ids(int64_t N, int64_t C, const int64_t* __restrict__ off, int* __restrict__ cid) {
    const int64_t k = blockIdx.x * int64_t(CB) + threadIdx.x;
    if (k >= N) return;
    cid[k] = int(clump_of(k, nullptr, off, C));
}

// sorted clump key of every point: its clump, or a value no other point has
// (-2 - caller index) for points outside every clump
__global__ void k_clump_sorted(int64_t N, const int* __restrict__ perm, const int* __restrict__ cid,
                               int* __restrict__ cid_s) {
    const int64_t i = blockIdx.x * int64_t(CB) + threadIdx.x;
    if (i >= N) return;
    const int j = perm[i];
    const int c = cid[j];
    cid_s[i] = c >= 0 ? c : -2 - j;
}

unsigned nblocks(int64_t n) { return unsigned((n + CB - 1) / CB); }

// The fixed scratch of kifmm_clump_reduce_noalloc: the segment partials of
// the reduction.  Every slot a call reads is written earlier by the same
// call, so nothing needs clearing; calls that overlap on one device share it
// and race.
__device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t clump_scratch_bytes(int64_t N, int nv) { return size_t(nblocks(N)) * 2 * nv * sizeof(double); }

void* noalloc_scratch() {
    int dev = 0;
    KIFMM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error(KIFMM_ERR_STATE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        // the host-side name of the array is not a device address: look the
        // device copy up once, with this device current
        void* p = nullptr;
        KIFMM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

void launch_clump_reduce(kifmm_plan* P, const float* q, const float* E, const int64_t* off, const int* cid, int64_t C,
                         const double* centers, double* F, double* T, double* part, hipStream_t s) {
    if (C <= 0) return;
    const int64_t N = P->N;
    hipLaunchKernelGGL(k_clump, dim3(nblocks(N)), dim3(CB), 0, s, N, C, off, cid, P->x64.as<double>(), q, E, centers,
                       F, T, part);
    hipLaunchKernelGGL(k_clump_fix<6>, dim3(nblocks(C)), dim3(CB), 0, s, C, N, off, part, F, T, P->status.as<int>(),
                       cid ? 0 : 1);
}

void launch_clump_backward(kifmm_plan* P, const float* q, const float* E, const int64_t* off, const int* cid,
                           int64_t C, const double* centers, const double* Fb, const double* Tb, float* qb,
                           float* Eb, float* xb, bool acc, double* Xb, double* part, hipStream_t s) {
    const int64_t N = P->N;
    hipLaunchKernelGGL(k_clump_bwd, dim3(nblocks(N)), dim3(CB), 0, s, N, C, off, cid, P->x64.as<double>(), q, E,
                       centers, Fb, Tb, qb, Eb, xb, acc ? 1 : 0, Xb, part);
    if (C > 0 && (Xb || !cid))
        hipLaunchKernelGGL(k_clump_fix<3>, dim3(nblocks(C)), dim3(CB), 0, s, C, N, off, part, Xb, nullptr,
                           P->status.as<int>(), cid ? 0 : 1);
}

void launch_clump_ids(kifmm_plan* P, hipStream_t s) {
    if (P->clumps <= 0) return;
    P->cid_s.ensure(size_t(P->N) * 4);
    hipLaunchKernelGGL(k_clump_sorted, dim3(nblocks(P->N)), dim3(CB), 0, s, P->N, P->perm.as<int>(), P->cid.as<int>(),
                       P->cid_s.as<int>());
}

void set_clump_ids(kifmm_plan* P, const int64_t* off_dev, int64_t C, hipStream_t s) {
    P->cid.ensure(size_t(P->N) * 4);
    hipLaunchKernelGGL(k_clump_ids, dim3(nblocks(P->N)), dim3(CB), 0, s, P->N, C, off_dev, P->cid.as<int>());
}

}  // namespace kifmm
