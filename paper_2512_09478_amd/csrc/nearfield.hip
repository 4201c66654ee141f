// Near field (Section 2.2, last step: the contributions of points in the near
// zone), written sorted as a float4 per point; the leaf-evaluation kernel adds
// it to the far field and writes the caller-order outputs.
//
// Work items of at most 64 targets of one leaf, launched heaviest first.  An
// item with 16 or more targets gives each of its four waves a quarter of the
// targets and all of the sources; a smaller item gives every wave all of its
// targets and every fourth group of sources.  Inside a wave a target has
// S = floor(64 / targets of the wave) consecutive lanes that split the
// sources, so at least 60 of the 64 lanes work; the lane partial sums are
// combined by a shuffle tree inside the group of S lanes and, for a small
// item, over the waves, both in a fixed order.
// The points of the U-list source leaves are streamed through LDS as float4
// (x, y, z, q) in global FP32 coordinates, many leaves per batch, so every
// pair difference is a correctly rounded FP32
// subtraction of the input coordinates.  Pairs at distance exactly zero (the
// self pair, coincident points) are skipped.  The forward kernel counts
// 20 FLOP per pair (3 sub, 5 for r^2, rsqrt, 4 for q/r and q/r^3, 7 for the
// four sums).
#include <math.h>

#include "common.h"

namespace kifmm {

namespace {

constexpr int NF_STAGE = 512;   // source points staged per batch

__global__ void k_gather(int64_t N, const float4* __restrict__ xs, const int* __restrict__ perm,
                         const float* __restrict__ q, float4* __restrict__ pts) {
    int64_t i = blockIdx.x * int64_t(256) + threadIdx.x;
    if (i >= N) return;
    float4 x = xs[i];
    x.w = q ? q[perm[i]] : 0.f;
    pts[i] = x;
}

__global__ void k_gather_adj(int64_t N, const int* __restrict__ perm, const float* __restrict__ gu,
                             const float* __restrict__ ge, float4* __restrict__ src2) {
    int64_t i = blockIdx.x * int64_t(256) + threadIdx.x;
    if (i >= N) return;
    int j = perm[i];
    src2[i] = make_float4(gu ? gu[j] : 0.f, ge ? ge[3 * size_t(j)] : 0.f, ge ? ge[3 * size_t(j) + 1] : 0.f,
                          ge ? ge[3 * size_t(j) + 2] : 0.f);
}

__device__ inline float rsq(float r2) { return r2 > 0.f ? __frsqrt_rn(r2) : 0.f; }

// Lane map of a work item (first target `first`, nt targets, 1 <= nt <= 64).
struct NearMap {
    int S;         // lanes per target in this wave (4 .. 64)
    int slice;     // this lane's place among them
    int i;         // target (sorted index)
    int j0, dj;    // staged sources j0, j0 + dj, ...
    bool act;      // the lane serves a target
    bool split;    // the waves split the sources (small item): sum over waves
};

__device__ inline NearMap near_map(int first, int nt) {
    NearMap m;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    m.split = nt < 16;
    const int per = m.split ? nt : (nt + 3) / 4;   // targets per wave
    const int t0 = m.split ? 0 : w * per;
    const int ntw = min(per, nt - t0);              // >= 1: nt - 3 ceil(nt/4) > 0 for nt >= 16
    m.S = 64 / ntw;
    m.slice = lane % m.S;
    const int tl = lane / m.S;
    m.act = tl < ntw;
    m.i = first + t0 + tl;
    m.j0 = m.split ? w * m.S + m.slice : m.slice;
    m.dj = m.split ? 4 * m.S : m.S;
    return m;
}

// Calls f(j) for this lane's staged sources j = j0, j0 + dj, ... below m.
// Every lane of the wave has T = ceil(m / dj) or T - 1 of them (j0 < dj), and
// its first T - 1 are below m: those steps run without a bounds check and
// with a wave-uniform trip count, only the last one is checked.
template <int UNROLL, class F>
__device__ inline void for_sources(const NearMap& nm, int m, F f) {
    const int T = __builtin_amdgcn_readfirstlane((m + nm.dj - 1) / nm.dj);
    int j = nm.j0;
#pragma unroll UNROLL
    for (int st = 0; st < T - 1; ++st, j += nm.dj) f(j);
    if (T > 0 && j < m) f(j);
}

// Sum over the S lanes of a target (lanes [g S, g S + S) of the wave); the
// first lane of the group ends with the total.
__device__ inline float group_sum(float v, int slice, int S) {
    for (int off = 1; off < S; off <<= 1) {
        const float t = __shfl_down(v, off, 64);
        if (slice + off < S) v += t;
    }
    return v;
}

// Stream the points of U(b) through LDS, all four waves staging together;
// calls body(m) after each batch of m staged points.  Block-uniform control.
// A periodic image of a leaf is staged moved by its shift times the cell side.
// With `ckey` the sources' clump keys are staged into shk as well.
template <class Body>
__device__ inline void stream_sources(const int* __restrict__ uoff, const int* __restrict__ uidx,
                                      const int2* __restrict__ range, int b, const float4* __restrict__ pts,
                                      const float4* __restrict__ src2, float cell, float4* sh, float4* sh2,
                                      Body body, const int* __restrict__ ckey = nullptr, int* shk = nullptr) {
    int k = uoff[b];
    const int kend = uoff[b + 1];
    int pos = 0;
    while (k < kend) {
        __syncthreads();
        int m = 0;
        while (k < kend && m < NF_STAGE) {
            const int e = uidx[k];
            const int2 ra = range[img_box(e)];
            int sx, sy, sz;
            img_shift(e, sx, sy, sz);
            const float ox = sx * cell, oy = sy * cell, oz = sz * cell;
            const int take = min(ra.y - ra.x - pos, NF_STAGE - m);
            for (int q = threadIdx.x; q < take; q += 256) {
                const float4 p = pts[ra.x + pos + q];
                sh[m + q] = make_float4(p.x + ox, p.y + oy, p.z + oz, p.w);
                if (src2) sh2[m + q] = src2[ra.x + pos + q];
                if (ckey) shk[m + q] = ckey[ra.x + pos + q];
            }
            m += take;
            pos += take;
            if (ra.x + pos == ra.y) {
                ++k;
                pos = 0;
            }
        }
        __syncthreads();
        body(m);
    }
}

// Sum NV per-lane values over the four waves in a fixed order (wave 0 ends
// with the totals).
template <int NV>
__device__ inline void wave_reduce(float (&v)[NV], float (*red)[NV][64]) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) red[w][q][lane] = v[q];
    __syncthreads();
    if (w == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = ((red[0][q][lane] + red[1][q][lane]) + red[2][q][lane]) + red[3][q][lane];
}

// Totals of an item's lane partials; true on the lane that writes them.
// Block-uniform (m.split depends on the item only).
template <int NV>
__device__ inline bool near_finish(float (&v)[NV], const NearMap& m, float (*red)[NV][64]) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = group_sum(v[q], m.slice, m.S);
    if (!m.split) return m.act && m.slice == 0;
    wave_reduce<NV>(v, red);
    return (threadIdx.x >> 6) == 0 && m.act && m.slice == 0;
}

// Work item = (leaf, first target): up to 64 targets, lanes as in near_map.
// EXCL: pairs whose clump keys (ckey, sorted) are equal are left out, which
// drops the pairs of pebbles of one clump and the self pair.
template <bool EXCL>
__global__ __launch_bounds__(256) void k_p2p(const int2* __restrict__ items, int n_items, const int2* __restrict__ range,
                                             const int* __restrict__ uoff, const int* __restrict__ uidx,
                                             const float4* __restrict__ pts, float cst, float cell,
                                             float4* __restrict__ nearv, const int* __restrict__ ckey) {
    __shared__ float4 sh[NF_STAGE];
    __shared__ int shk[EXCL ? NF_STAGE : 1];
    __shared__ float red[4][4][64];
    // the grid strides over the items (launched with one block per item)
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int2 it = items[item];
        const int b = it.x;
        const int nt = min(64, range[b].y - it.y);
        const NearMap nm = near_map(it.y, nt);
        const int i = nm.i;
        const bool act = nm.act;
        const float4 x = act ? pts[i] : make_float4(0, 0, 0, 0);
        const int ck = (EXCL && act) ? ckey[i] : 0;
        float v[4] = {0.f, 0.f, 0.f, 0.f};   // u, ex, ey, ez
        stream_sources(uoff, uidx, range, b, pts, nullptr, cell, sh, nullptr, [&](int m) {
            for_sources<4>(nm, m, [&](int j) {
                const float4 y = sh[j];
                const float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z;
                float ri = rsq(dx * dx + dy * dy + dz * dz);
                if (EXCL) ri = shk[j] != ck ? ri : 0.f;
                const float qr = y.w * ri;
                const float qr3 = qr * ri * ri;
                v[0] += qr;
                v[1] += qr3 * dx;
                v[2] += qr3 * dy;
                v[3] += qr3 * dz;
            });
        }, EXCL ? ckey : nullptr, shk);
        if (near_finish<4>(v, nm, red)) nearv[i] = make_float4(cst * v[0], cst * v[1], cst * v[2], cst * v[3]);
    }
}

// Near field of monopoles q_j and dipoles m_j (src2 = (q, m) sorted):
//   u += q_j/r - m_j.r/r^3,  E = -grad u += r (q_j/r^3 - 3 m_j.r/r^5) + m_j/r^3.
__global__ __launch_bounds__(256) void k_p2p_dip(const int2* __restrict__ items, int n_items,
                                                 const int2* __restrict__ range, const int* __restrict__ uoff,
                                                 const int* __restrict__ uidx, const float4* __restrict__ pts,
                                                 const float4* __restrict__ src2, float cst, float cell,
                                                 float4* __restrict__ nearv) {
    __shared__ float4 sh[NF_STAGE];
    __shared__ float4 sh2[NF_STAGE];
    __shared__ float red[4][4][64];
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int2 it = items[item];
        const int b = it.x;
        const int nt = min(64, range[b].y - it.y);
        const NearMap nm = near_map(it.y, nt);
        const int i = nm.i;
        const bool act = nm.act;
        const float4 x = act ? pts[i] : make_float4(0, 0, 0, 0);
        float v[4] = {0.f, 0.f, 0.f, 0.f};   // u, ex, ey, ez
        stream_sources(uoff, uidx, range, b, pts, src2, cell, sh, sh2, [&](int m) {
            for_sources<2>(nm, m, [&](int j) {
                const float4 y = sh[j];
                const float4 bj = sh2[j];
                const float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z;
                const float ri = rsq(dx * dx + dy * dy + dz * dz);
                const float ri2 = ri * ri;
                const float ri3 = ri2 * ri;
                // with c = m.r/r^2: u term (q - c)/r, radial field (q - 3c)/r^3
                const float c = (dx * bj.y + dy * bj.z + dz * bj.w) * ri2;
                v[0] += ri * (bj.x - c);
                const float gh = ri3 * (bj.x - 3.f * c);
                v[1] += gh * dx + bj.y * ri3;
                v[2] += gh * dy + bj.z * ri3;
                v[3] += gh * dz + bj.w * ri3;
            });
        });
        if (near_finish<4>(v, nm, red)) nearv[i] = make_float4(cst * v[0], cst * v[1], cst * v[2], cst * v[3]);
    }
}

// Near field with the field gradient, of monopoles (src2.x, or pts.w without
// src2) and dipoles (src2.yzw): u, E and dE_a/dx_b = -Hess u, the dipole
// part of the Hessian being 3 (m_a r_b + m_b r_a + (m.r) delta_ab)/r^5
// - 15 (m.r) r_a r_b / r^7.  (u, E) go to nearv, dE/dx (xx yy zz xy xz yz)
// to nearg.
template <bool DIP>
__global__ __launch_bounds__(256) void k_p2p_grad(const int2* __restrict__ items, int n_items,
                                                  const int2* __restrict__ range, const int* __restrict__ uoff,
                                                  const int* __restrict__ uidx, const float4* __restrict__ pts,
                                                  const float4* __restrict__ src2, float cst, float cell,
                                                  float4* __restrict__ nearv, float* __restrict__ nearg) {
    __shared__ float4 sh[NF_STAGE];
    __shared__ float4 sh2[DIP ? NF_STAGE : 1];
    __shared__ float red[4][10][64];
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int2 it = items[item];
        const int b = it.x;
        const int nt = min(64, range[b].y - it.y);
        const NearMap nm = near_map(it.y, nt);
        const int i = nm.i;
        const bool act = nm.act;
        const float4 x = act ? pts[i] : make_float4(0, 0, 0, 0);
        float v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // u, E xyz, dE/dx xx yy zz xy xz yz
        stream_sources(uoff, uidx, range, b, pts, DIP ? src2 : nullptr, cell, sh, sh2, [&](int m) {
            for_sources<DIP ? 2 : 4>(nm, m, [&](int j) {
                const float4 y = sh[j];
                const float d0 = x.x - y.x, d1 = x.y - y.y, d2 = x.z - y.z;
                const float ri = rsq(d0 * d0 + d1 * d1 + d2 * d2);
                const float ri2 = ri * ri;
                const float ri3 = ri2 * ri;
                if constexpr (!DIP) {
                    // charge q: u = q/r, E = g d, dE_a/dx_c = g delta_ac - 3 g d_a d_c / r^2, g = q/r^3
                    const float g = y.w * ri3;
                    const float c = -3.f * g * ri2;
                    v[0] += y.w * ri;
                    v[1] += g * d0;
                    v[2] += g * d1;
                    v[3] += g * d2;
                    const float e0 = c * d0, e1 = c * d1, e2 = c * d2;
                    v[4] += e0 * d0 + g;
                    v[5] += e1 * d1 + g;
                    v[6] += e2 * d2 + g;
                    v[7] += e0 * d1;
                    v[8] += e0 * d2;
                    v[9] += e1 * d2;
                } else {
                    // charge q and dipole m (u += q/r - m.d/r^3): with t = 3 (m.d)/r^5,
                    // E = gh d + m/r^3, gh = q/r^3 - t, and
                    // dE_a/dx_c = coef d_a d_c - p_a d_c - p_c d_a + gh delta_ac,
                    // coef = 5 t/r^2 - 3 q/r^5, p = 3 m/r^5
                    const float4 bj = sh2[j];
                    const float ri5 = ri3 * ri2;
                    const float mr = d0 * bj.y + d1 * bj.z + d2 * bj.w;
                    const float t = 3.f * mr * ri5;
                    const float gh = bj.x * ri3 - t;
                    v[0] += bj.x * ri - mr * ri3;
                    v[1] += gh * d0 + bj.y * ri3;
                    v[2] += gh * d1 + bj.z * ri3;
                    v[3] += gh * d2 + bj.w * ri3;
                    const float coef = 5.f * t * ri2 - 3.f * bj.x * ri5;
                    const float p0 = 3.f * ri5 * bj.y, p1 = 3.f * ri5 * bj.z, p2 = 3.f * ri5 * bj.w;
                    // e_a = coef d_a - p_a, so that dE_a/dx_c = e_a d_c - p_c d_a (+ gh on the diagonal)
                    const float e0 = coef * d0 - p0, e1 = coef * d1 - p1, e2 = coef * d2 - p2;
                    v[4] += (e0 - p0) * d0 + gh;
                    v[5] += (e1 - p1) * d1 + gh;
                    v[6] += (e2 - p2) * d2 + gh;
                    v[7] += e0 * d1 - p1 * d0;
                    v[8] += e0 * d2 - p2 * d0;
                    v[9] += e1 * d2 - p2 * d1;
                }
            });
        });
        if (near_finish<10>(v, nm, red)) {
            nearv[i] = make_float4(cst * v[0], cst * v[1], cst * v[2], cst * v[3]);
#pragma unroll
            for (int k = 0; k < 6; ++k) nearg[6 * size_t(i) + k] = cst * v[4 + k];
        }
    }
}

// Backward near field, summed directly as the near part of the combination
//   qbar_k = psi_k,  xbar_k = -ubar_k E_k - H_k Ebar_k - q_k E_psi,k
// where E, H come from the charges q and psi, E_psi from monopoles ubar and
// dipoles Ebar (psi = sum ubar K - Ebar . G).
// Eight blocks per CU: the wave reduction of a small item reuses the staging
// LDS (its first barrier follows the item's last batch), so a block holds
// 16 KB, and the register budget is 64.
template <bool EXCL>
__global__ __launch_bounds__(256, 8) void k_p2p_bwd(const int2* __restrict__ items, int n_items,
                                                    const int2* __restrict__ range, const int* __restrict__ uoff,
                                                    const int* __restrict__ uidx, const float4* __restrict__ pts,
                                                    const float4* __restrict__ src2, float cst, float cell,
                                                    float4* __restrict__ nearv, const int* __restrict__ ckey) {
    __shared__ float4 stage[2 * NF_STAGE];
    __shared__ int shk[EXCL ? NF_STAGE : 1];
    float4* sh = stage;
    float4* sh2 = stage + NF_STAGE;
    static_assert(sizeof(float) * 4 * 9 * 64 <= sizeof(float4) * 2 * NF_STAGE, "reduction fits the staging");
    float(*red)[9][64] = reinterpret_cast<float(*)[9][64]>(stage);
    // the grid strides over the items (launched with one block per item)
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int2 it = items[item];
        const int b = it.x;
        const int nt = min(64, range[b].y - it.y);
        const NearMap nm = near_map(it.y, nt);
        const int i = nm.i;
        const bool act = nm.act;
        const float4 x = act ? pts[i] : make_float4(0, 0, 0, 0);
        const float4 a = act ? src2[i] : make_float4(0, 0, 0, 0);
        // The adjoint combination xbar_k = -ubar_k E_k - H_k Ebar_k - q_k E_psi,k
        // is summed pair by pair (r = x_k - y_j, c applied at the end):
        //   xbar += r [-(ubar_k q_j + q_k ubar_j)/r^3 - 3 (q_j r.Ebar_k - q_k r.Ebar_j)/r^5]
        //           + (q_j Ebar_k - q_k Ebar_j)/r^3,
        // with the target's Ebar_k taken out of the sum: v = (X xyz, S, T xyz, psi)
        // and xbar = X + S Ebar_k - q_k T;  qbar = psi = sum ubar_j/r - r.Ebar_j/r^3.
        // psi is kept as its two sums (v[7] ubar_j / r, v[8] r.Ebar_j / r^3)
        float v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        const float uk = a.x, qk = x.w;
        const int ck = (EXCL && act) ? ckey[i] : 0;
        stream_sources(uoff, uidx, range, b, pts, src2, cell, sh, sh2, [&](int m) {
            for_sources<1>(nm, m, [&](int j) {
                const float4 y = sh[j];
                const float4 bj = sh2[j];
                const float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z;
                float ri = rsq(dx * dx + dy * dy + dz * dz);
                if (EXCL) ri = shk[j] != ck ? ri : 0.f;
                const float ri2 = ri * ri;
                const float ri3 = ri2 * ri;
                const float rk = dx * a.y + dy * a.z + dz * a.w;
                const float rj = dx * bj.y + dy * bj.z + dz * bj.w;
                const float t1 = uk * y.w + qk * bj.x;
                const float t2 = y.w * rk - qk * rj;
                // -(t1 / r^3 + 3 t2 / r^5)
                const float coef = -ri3 * (t1 + 3.f * (ri2 * t2));
                v[0] += coef * dx;
                v[1] += coef * dy;
                v[2] += coef * dz;
                v[3] += y.w * ri3;
                v[4] += bj.y * ri3;
                v[5] += bj.z * ri3;
                v[6] += bj.w * ri3;
                v[7] += bj.x * ri;
                v[8] += rj * ri3;
            });
        }, EXCL ? ckey : nullptr, shk);
        if (near_finish<9>(v, nm, red))
            nearv[i] = make_float4(cst * (v[0] + v[3] * a.y - qk * v[4]), cst * (v[1] + v[3] * a.z - qk * v[5]),
                                   cst * (v[2] + v[3] * a.w - qk * v[6]), cst * (v[7] - v[8]));
    }
}

// Stokeslet sources: pass 0 sets pts.w = f_x, src2 = (f_y, 0, 0, 0) and the
// sorted forces stk = (f_x, f_y, f_z, 0); pass 1 sets pts.w = f_z.  The
// fourth harmonic charge, (x - c) . f about each box's centre c, is formed
// from stk where a box's sources are summed.
__global__ void k_gather_stokes(int64_t N, const float4* __restrict__ xs, const int* __restrict__ perm,
                                const float* __restrict__ f, int pass, float4* __restrict__ pts,
                                float4* __restrict__ src2, float4* __restrict__ stk) {
    int64_t i = blockIdx.x * int64_t(256) + threadIdx.x;
    if (i >= N) return;
    const size_t j = size_t(perm[i]);
    const float fx = f[3 * j], fy = f[3 * j + 1], fz = f[3 * j + 2];
    float4 x = xs[i];
    if (pass == 0) {
        x.w = fx;
        src2[i] = make_float4(fy, 0.f, 0.f, 0.f);
        stk[i] = make_float4(fx, fy, fz, 0.f);
    } else {
        x.w = fz;
    }
    pts[i] = x;
}

// Near field of point forces (the Stokeslet): u += f/r + (r.f) r/r^3 over
// the near lists, pairs at distance zero skipped; positions from xs, forces
// from stk (sorted); written as cst * u to out (sorted), with the unscaled sum
// of (r.f)/r^3 (the near part of the pressure, times 4 pi) in the fourth
// component.
__global__ __launch_bounds__(256) void k_p2p_stokes(const int2* __restrict__ items, int n_items,
                                                    const int2* __restrict__ range, const int* __restrict__ uoff,
                                                    const int* __restrict__ uidx, const float4* __restrict__ xs,
                                                    const float4* __restrict__ stk, float cst,
                                                    float4* __restrict__ out) {
    __shared__ float4 sh[NF_STAGE];
    __shared__ float4 sh2[NF_STAGE];
    __shared__ float red[4][4][64];
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int2 it = items[item];
        const int b = it.x;
        const int nt = min(64, range[b].y - it.y);
        const NearMap nm = near_map(it.y, nt);
        const int i = nm.i;
        const float4 x = nm.act ? xs[i] : make_float4(0, 0, 0, 0);
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        stream_sources(uoff, uidx, range, b, xs, stk, 0.f, sh, sh2, [&](int m) {
            for_sources<1>(nm, m, [&](int j) {
                const float4 y = sh[j];
                const float4 fj = sh2[j];
                const float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z;
                const float ri = rsq(dx * dx + dy * dy + dz * dz);
                const float t = (dx * fj.x + dy * fj.y + dz * fj.z) * ri * ri * ri;
                v[0] += fj.x * ri + t * dx;
                v[1] += fj.y * ri + t * dy;
                v[2] += fj.z * ri + t * dz;
                v[3] += t;
            });
        });
        if (near_finish<4>(v, nm, red)) out[i] = make_float4(cst * v[0], cst * v[1], cst * v[2], v[3]);
    }
}

}  // namespace

void launch_gather(kifmm_plan* P, const float* charges, const float* gpot, const float* gfield, bool adjoint,
                   hipStream_t s, bool points) {
    const int64_t N = P->N;
    if (charges || points) {
        P->pts.ensure(size_t(N) * 16);
        hipLaunchKernelGGL(k_gather, dim3(unsigned((N + 255) / 256)), dim3(256), 0, s, N, P->xs.as<float4>(),
                           P->perm.as<int>(), charges, P->pts.as<float4>());
    }
    if (adjoint) {
        P->src2.ensure(size_t(N) * 16);
        hipLaunchKernelGGL(k_gather_adj, dim3(unsigned((N + 255) / 256)), dim3(256), 0, s, N, P->perm.as<int>(), gpot,
                           gfield, P->src2.as<float4>());
    }
}

void launch_p2p_forward(kifmm_plan* P, hipStream_t s, bool excl) {
    if (excl)
        hipLaunchKernelGGL(k_p2p<true>, dim3(unsigned(P->n_items)), dim3(256), 0, s, P->items_near.as<int2>(),
                           int(P->n_items), P->bx_range.as<int2>(), P->n_off.as<int>(), P->n_idx.as<int>(),
                           P->pts.as<float4>(), float(P->c), float(P->side), P->nearv.as<float4>(),
                           (const int*)P->cid_s.as<int>());
    else
        hipLaunchKernelGGL(k_p2p<false>, dim3(unsigned(P->n_items)), dim3(256), 0, s, P->items_near.as<int2>(),
                           int(P->n_items), P->bx_range.as<int2>(), P->n_off.as<int>(), P->n_idx.as<int>(),
                           P->pts.as<float4>(), float(P->c), float(P->side), P->nearv.as<float4>(),
                           (const int*)nullptr);
}

void launch_gather_stokes(kifmm_plan* P, const float* forces, int pass, hipStream_t s) {
    const int64_t N = P->N;
    P->pts.ensure(size_t(N) * 16);
    P->src2.ensure(size_t(N) * 16);
    P->stk.ensure(size_t(N) * 16);
    hipLaunchKernelGGL(k_gather_stokes, dim3(unsigned((N + 255) / 256)), dim3(256), 0, s, N, P->xs.as<float4>(),
                       P->perm.as<int>(), forces, pass, P->pts.as<float4>(), P->src2.as<float4>(),
                       P->stk.as<float4>());
}

void launch_p2p_stokes(kifmm_plan* P, double viscosity, hipStream_t s) {
    P->stk_near.ensure(size_t(P->N) * 16);
    // the Stokes cell is not periodic: no image shifts in the lists
    hipLaunchKernelGGL(k_p2p_stokes, dim3(unsigned(P->n_items)), dim3(256), 0, s, P->items_near.as<int2>(),
                       int(P->n_items), P->bx_range.as<int2>(), P->n_off.as<int>(), P->n_idx.as<int>(),
                       P->xs.as<float4>(), P->stk.as<float4>(), float(1.0 / (8.0 * M_PI * viscosity)),
                       P->stk_near.as<float4>());
}

void launch_p2p_dipoles(kifmm_plan* P, hipStream_t s) {
    hipLaunchKernelGGL(k_p2p_dip, dim3(unsigned(P->n_items)), dim3(256), 0, s, P->items_near.as<int2>(),
                       int(P->n_items), P->bx_range.as<int2>(), P->n_off.as<int>(), P->n_idx.as<int>(),
                       P->pts.as<float4>(), P->src2.as<float4>(), float(P->c), float(P->side), P->nearv.as<float4>());
}

void launch_p2p_gradient(kifmm_plan* P, bool dipoles, hipStream_t s) {
    P->nearg.ensure(size_t(P->N) * 24);
    if (dipoles)
        hipLaunchKernelGGL(k_p2p_grad<true>, dim3(unsigned(P->n_items)), dim3(256), 0, s, P->items_near.as<int2>(),
                           int(P->n_items), P->bx_range.as<int2>(), P->n_off.as<int>(), P->n_idx.as<int>(),
                           P->pts.as<float4>(), P->src2.as<float4>(), float(P->c), float(P->side),
                           P->nearv.as<float4>(), P->nearg.as<float>());
    else
        hipLaunchKernelGGL(k_p2p_grad<false>, dim3(unsigned(P->n_items)), dim3(256), 0, s, P->items_near.as<int2>(),
                           int(P->n_items), P->bx_range.as<int2>(), P->n_off.as<int>(), P->n_idx.as<int>(),
                           P->pts.as<float4>(), (const float4*)nullptr, float(P->c), float(P->side),
                           P->nearv.as<float4>(), P->nearg.as<float>());
}

void launch_p2p_backward(kifmm_plan* P, hipStream_t s, bool excl) {
    if (excl)
        hipLaunchKernelGGL(k_p2p_bwd<true>, dim3(unsigned(P->n_items)), dim3(256), 0, s, P->items_near.as<int2>(),
                           int(P->n_items), P->bx_range.as<int2>(), P->n_off.as<int>(), P->n_idx.as<int>(),
                           P->pts.as<float4>(), P->src2.as<float4>(), float(P->c), float(P->side),
                           P->nearv.as<float4>(), (const int*)P->cid_s.as<int>());
    else
        hipLaunchKernelGGL(k_p2p_bwd<false>, dim3(unsigned(P->n_items)), dim3(256), 0, s, P->items_near.as<int2>(),
                           int(P->n_items), P->bx_range.as<int2>(), P->n_off.as<int>(), P->n_idx.as<int>(),
                           P->pts.as<float4>(), P->src2.as<float4>(), float(P->c), float(P->side),
                           P->nearv.as<float4>(), (const int*)nullptr);
}

}  // namespace kifmm
