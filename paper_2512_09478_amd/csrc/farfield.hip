// Far field of the KIFMM sweep (Section 2.2, steps two to four): P2M, the
// upward M2M + check-to-equivalent apply, P2L (X list), M2L (V list), L2L +
// downward check-to-equivalent apply, and the leaf evaluation L2P + M2P.
//
// Normalised quantities.  For a box of side w with centre c a point enters as
// x' = (x - c)/w; check potentials are stored multiplied by w/c (c the kernel
// constant), so with K1(r) = 1/|r| every operator is the same matrix at every
// level and equivalent densities are in charge units.  Outputs are multiplied
// by c/w (potential), c/w^2 (field) and c/w^3 (Hessian).
//
// The dense contractions (M2M, M2L, L2L and the factored check-to-equivalent
// maps) run on MFMA: a wave owns 16 target boxes (one 16-column block) and all
// NP padded rows; the operator (row-major, NP x NP) is the A operand read from
// L2, the gathered source densities are the B operand.  With
// v_mfma_f32_16x16x4_f32 a lane holds A[row = lane%16][k = lane/16] and
// B[k = lane/16][col = lane%16], and the accumulator holds
// D[4 (lane/16) + r][lane%16]; each lane loads 8 consecutive k values and the
// eight MFMAs of a 32-wide k chunk take one of them each, which permutes the
// k order but not the sum.  A result in accumulator layout is itself the B
// operand of a following product (k = 16 rb + 4 g + r), which chains the two
// factors of a check-to-equivalent map without leaving registers.  The split
// path uses v_mfma_f32_16x16x32_bf16 with operands hi = bf16(x),
// lo = bf16(x - hi) and D += Ahi Bhi + Ahi Blo + Alo Bhi in FP32.
#include <algorithm>

#include "common.h"

namespace kifmm {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int WAVES = 4;

struct BoxGeom {
    double lo[3];
    double side;
};

__device__ inline void box_frame(const BoxGeom& g, int4 a, float c[3], float& invw, float& w) {
    double wd = ldexp(g.side, -a.w);
    c[0] = float(g.lo[0] + (double(a.x) + 0.5) * wd);
    c[1] = float(g.lo[1] + (double(a.y) + 0.5) * wd);
    c[2] = float(g.lo[2] + (double(a.z) + 0.5) * wd);
    w = float(wd);
    invw = float(ldexp(1.0, a.w) / g.side);
}

__device__ inline float rsq(float r2) { return r2 > 0.f ? __frsqrt_rn(r2) : 0.f; }

// ------------------------------------------------------------------ MFMA engine
template <int NP>
__device__ inline void zero_acc(v4f* acc) {
#pragma unroll
    for (int rb = 0; rb < NP / 16; ++rb) acc[rb] = v4f{0.f, 0.f, 0.f, 0.f};
}

template <int NP>
__device__ inline void load_acc(v4f* acc, const float* __restrict__ col, int lane) {
    const int g = lane >> 4;
#pragma unroll
    for (int rb = 0; rb < NP / 16; ++rb) {
        if (col) {
            float4 v = *reinterpret_cast<const float4*>(col + rb * 16 + 4 * g);
            acc[rb] = v4f{v.x, v.y, v.z, v.w};
        } else {
            acc[rb] = v4f{0.f, 0.f, 0.f, 0.f};
        }
    }
}

template <int NP>
__device__ inline void store_acc(const v4f* acc, float* __restrict__ col, int lane) {
    const int g = lane >> 4;
    if (!col) return;
#pragma unroll
    for (int rb = 0; rb < NP / 16; ++rb)
        *reinterpret_cast<float4*>(col + rb * 16 + 4 * g) = make_float4(acc[rb][0], acc[rb][1], acc[rb][2], acc[rb][3]);
}

// acc += A * b, A row-major NP x NP (FP32), b this lane's source column (or null = 0)
template <int NP>
__device__ inline void gemm_f32(v4f* acc, const float* __restrict__ A, const float* __restrict__ b, int lane) {
    const int g = lane >> 4, r = lane & 15;
    for (int kc = 0; kc < NP; kc += 32) {
        float bv[8];
        if (b) {
            float4 b0 = *reinterpret_cast<const float4*>(b + kc + 8 * g);
            float4 b1 = *reinterpret_cast<const float4*>(b + kc + 8 * g + 4);
            bv[0] = b0.x; bv[1] = b0.y; bv[2] = b0.z; bv[3] = b0.w;
            bv[4] = b1.x; bv[5] = b1.y; bv[6] = b1.z; bv[7] = b1.w;
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) bv[i] = 0.f;
        }
#pragma unroll
        for (int rb = 0; rb < NP / 16; ++rb) {
            const float* ap = A + size_t(rb * 16 + r) * NP + kc + 8 * g;
            float4 a0 = *reinterpret_cast<const float4*>(ap);
            float4 a1 = *reinterpret_cast<const float4*>(ap + 4);
            v4f c = acc[rb];
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.x, bv[0], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.y, bv[1], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.z, bv[2], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.w, bv[3], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.x, bv[4], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.y, bv[5], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.z, bv[6], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.w, bv[7], c, 0, 0, 0);
            acc[rb] = c;
        }
    }
}

// acc += A * b with A and b split into bf16 hi/lo (A pre-split, b split here)
template <int NP>
__device__ inline void gemm_bf16x3(v4f* acc, const __bf16* __restrict__ Ahi, const __bf16* __restrict__ Alo,
                                   const float* __restrict__ b, int lane) {
    const int g = lane >> 4, r = lane & 15;
    for (int kc = 0; kc < NP; kc += 32) {
        v8bf bh, bl;
        if (b) {
            float4 b0 = *reinterpret_cast<const float4*>(b + kc + 8 * g);
            float4 b1 = *reinterpret_cast<const float4*>(b + kc + 8 * g + 4);
            float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                __bf16 h = (__bf16)bv[i];
                bh[i] = h;
                bl[i] = (__bf16)(bv[i] - (float)h);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                bh[i] = (__bf16)0.f;
                bl[i] = (__bf16)0.f;
            }
        }
#pragma unroll
        for (int rb = 0; rb < NP / 16; ++rb) {
            size_t off = size_t(rb * 16 + r) * NP + kc + 8 * g;
            v8bf ah = *reinterpret_cast<const v8bf*>(Ahi + off);
            v8bf al = *reinterpret_cast<const v8bf*>(Alo + off);
            v4f c = acc[rb];
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
            acc[rb] = c;
        }
    }
}

// out += A * T, with T given in accumulator layout (row k = 16 rb + 4 g + r)
template <int NP>
__device__ inline void gemm_f32_chain(v4f* out, const float* __restrict__ A, const v4f* T, int lane) {
    const int g = lane >> 4, r = lane & 15;
#pragma unroll
    for (int ob = 0; ob < NP / 16; ++ob) {
        v4f c = out[ob];
        const float* ap = A + size_t(ob * 16 + r) * NP + 4 * g;
#pragma unroll
        for (int rb = 0; rb < NP / 16; ++rb) {
            float4 a = *reinterpret_cast<const float4*>(ap + rb * 16);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, T[rb][0], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, T[rb][1], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, T[rb][2], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, T[rb][3], c, 0, 0, 0);
        }
        out[ob] = c;
    }
}

// phi = Vm * (W1 * psi): the factored check-to-equivalent map on an accumulator
template <int NP>
__device__ inline void c2e_apply(v4f* acc, const float* __restrict__ W1, const float* __restrict__ Vm, int lane) {
    v4f t[NP / 16];
    zero_acc<NP>(t);
    gemm_f32_chain<NP>(t, W1, acc, lane);
    zero_acc<NP>(acc);
    gemm_f32_chain<NP>(acc, Vm, t, lane);
}

// ------------------------------------------------------------------ P2M / P2L
// Check potential of leaf points on a surface of box `b` (normalised):
// psi[i] = sum_j q_j K1(s_i - x'_j) - (1/w) Ebar_j . G1(s_i - x'_j)   (dipole part optional)
template <int NP>
__device__ void points_to_surface(float& acc, const float4* __restrict__ pts, const float4* __restrict__ src2,
                                  int j0, int j1, const float c[3], float invw, float4 s, bool active,
                                  float4* sh, float4* sh2) {
    for (int base = j0; base < j1; base += 256) {
        int m = min(256, j1 - base);
        __syncthreads();
        for (int k = threadIdx.x; k < m; k += blockDim.x) {
            float4 p = pts[base + k];
            sh[k] = make_float4((p.x - c[0]) * invw, (p.y - c[1]) * invw, (p.z - c[2]) * invw, p.w);
            if (src2) {
                float4 a = src2[base + k];
                sh2[k] = make_float4(a.x, a.y * invw, a.z * invw, a.w * invw);
            }
        }
        __syncthreads();
        if (active) {
            if (!src2) {
                for (int k = 0; k < m; ++k) {
                    float4 p = sh[k];
                    float dx = s.x - p.x, dy = s.y - p.y, dz = s.z - p.z;
                    acc += p.w * rsq(dx * dx + dy * dy + dz * dz);
                }
            } else {
                for (int k = 0; k < m; ++k) {
                    float4 p = sh[k];
                    float4 a = sh2[k];
                    float dx = s.x - p.x, dy = s.y - p.y, dz = s.z - p.z;
                    float ri = rsq(dx * dx + dy * dy + dz * dz);
                    float ri3 = ri * ri * ri;
                    acc += a.x * ri - (a.y * dx + a.z * dy + a.w * dz) * ri3;
                }
            }
        }
    }
}

template <int NP>
__global__ void k_p2m(const int* __restrict__ leaves, int nleaves, int b2, const int4* __restrict__ anchor,
                      const int2* __restrict__ range, const float4* __restrict__ pts,
                      const float4* __restrict__ src2, const float4* __restrict__ surf, int n, BoxGeom geo,
                      float* __restrict__ psi_u) {
    __shared__ float4 sh[256];
    __shared__ float4 sh2[256];
    int b = leaves[blockIdx.x];
    if (b < b2) return;   // leaves above level 2 have no far field
    int4 a = anchor[b];
    float c[3], invw, w;
    box_frame(geo, a, c, invw, w);
    int2 r = range[b];
    for (int i0 = 0; i0 < NP; i0 += blockDim.x) {
        int i = i0 + threadIdx.x;
        bool act = i < n;
        float4 s = act ? surf[NP + i] : make_float4(0, 0, 0, 0);   // upward check surface
        float acc = 0.f;
        points_to_surface<NP>(acc, pts, src2, r.x, r.y, c, invw, s, act, sh, sh2);
        if (i < NP) psi_u[size_t(b) * NP + i] = act ? acc : 0.f;
    }
}

template <int NP>
__global__ void k_p2l(const int* __restrict__ xboxes, const int* __restrict__ xoff, const int* __restrict__ xidx,
                      const int4* __restrict__ anchor, const int2* __restrict__ range,
                      const float4* __restrict__ pts, const float4* __restrict__ src2,
                      const float4* __restrict__ surf, int n, BoxGeom geo, float* __restrict__ psi_d) {
    __shared__ float4 sh[256];
    __shared__ float4 sh2[256];
    int b = xboxes[blockIdx.x];
    int4 a = anchor[b];
    float c[3], invw, w;
    box_frame(geo, a, c, invw, w);
    for (int i0 = 0; i0 < NP; i0 += blockDim.x) {
        int i = i0 + threadIdx.x;
        bool act = i < n;
        float4 s = act ? surf[i] : make_float4(0, 0, 0, 0);   // downward check surface
        float acc = 0.f;
        for (int k = xoff[b]; k < xoff[b + 1]; ++k) {
            int2 r = range[xidx[k]];
            points_to_surface<NP>(acc, pts, src2, r.x, r.y, c, invw, s, act, sh, sh2);
        }
        if (i < NP) psi_d[size_t(b) * NP + i] = act ? acc : 0.f;
    }
}

// ------------------------------------------------------------------ upward: M2M + UC2E
template <int NP>
__global__ __launch_bounds__(256) void k_up(int b0, int nb, const int2* __restrict__ child,
                                            const int* __restrict__ leafflag, const float* __restrict__ psi_u,
                                            float* __restrict__ phi_u, const float* __restrict__ m2m,
                                            const float* __restrict__ w1, const float* __restrict__ vm) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t0 = (blockIdx.x * WAVES + wave) * 16;
    if (t0 >= nb) return;
    const int t = t0 + (lane & 15) < nb ? b0 + t0 + (lane & 15) : -1;
    const bool leaf = t >= 0 && leafflag[t];
    v4f acc[NP / 16];
    load_acc<NP>(acc, leaf ? psi_u + size_t(t) * NP : nullptr, lane);
    int2 ch = (t >= 0 && !leaf) ? child[t] : make_int2(-1, 0);
    if (__ballot(ch.y != 0)) {
        for (int o = 0; o < 8; ++o) {
            int src = ((ch.y >> o) & 1) ? ch.x + __popc(ch.y & ((1 << o) - 1)) : -1;
            if (!__ballot(src >= 0)) continue;
            gemm_f32<NP>(acc, m2m + size_t(o) * NP * NP, src >= 0 ? phi_u + size_t(src) * NP : nullptr, lane);
        }
    }
    c2e_apply<NP>(acc, w1, vm, lane);
    store_acc<NP>(acc, t >= 0 ? phi_u + size_t(t) * NP : nullptr, lane);
}

// ------------------------------------------------------------------ M2L
struct TaskTable {
    int nlev;
    int first[kMaxLevels + 1];   // first block of level entry
    int level[kMaxLevels + 1];
    int nl_start[kMaxLevels + 1];   // parents (non-leaf boxes of level-1)
    int nl_count[kMaxLevels + 1];
    int groups[kMaxLevels + 1];     // groups of WAVES*16 parents
};

struct VOps {
    short op[8][kVPerOct];
};

template <int NP, bool SPLIT>
__global__ __launch_bounds__(256) void k_m2l(TaskTable tt, const int* __restrict__ nonleaf,
                                             const int2* __restrict__ child, const int* __restrict__ vdense,
                                             int b2, const VOps* __restrict__ vops,
                                             const float* __restrict__ phi_u, float* __restrict__ psi_d,
                                             const float* __restrict__ m2l, const __bf16* __restrict__ m2l_hi,
                                             const __bf16* __restrict__ m2l_lo) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int e = 0;
    while (e + 1 < tt.nlev && int(blockIdx.x) >= tt.first[e + 1]) ++e;
    int local = blockIdx.x - tt.first[e];
    int o = local % 8;
    int grp = local / 8;
    int slot = (grp * WAVES + wave) * 16 + (lane & 15);
    int t = -1;
    if (slot < tt.nl_count[e]) {
        int Pb = nonleaf[tt.nl_start[e] + slot];
        int2 ch = child[Pb];
        if ((ch.y >> o) & 1) t = ch.x + __popc(ch.y & ((1 << o) - 1));
    }
    if (!__ballot(t >= 0)) return;
    v4f acc[NP / 16];
    load_acc<NP>(acc, t >= 0 ? psi_d + size_t(t) * NP : nullptr, lane);
    const int* vrow = t >= 0 ? vdense + size_t(t - b2) * kVPerOct : nullptr;
    for (int j = 0; j < kVPerOct; ++j) {
        int src = vrow ? vrow[j] : -1;
        if (!__ballot(src >= 0)) continue;
        int m = vops->op[o][j];
        const float* bcol = src >= 0 ? phi_u + size_t(src) * NP : nullptr;
        if (SPLIT)
            gemm_bf16x3<NP>(acc, m2l_hi + size_t(m) * NP * NP, m2l_lo + size_t(m) * NP * NP, bcol, lane);
        else
            gemm_f32<NP>(acc, m2l + size_t(m) * NP * NP, bcol, lane);
    }
    store_acc<NP>(acc, t >= 0 ? psi_d + size_t(t) * NP : nullptr, lane);
}

// ------------------------------------------------------------------ downward: L2L + DC2E
template <int NP>
__global__ __launch_bounds__(256) void k_down(int nl_start, int nl_count, int has_l2l,
                                              const int* __restrict__ nonleaf, const int2* __restrict__ child,
                                              const float* __restrict__ psi_d, float* __restrict__ phi_d,
                                              const float* __restrict__ l2l, const float* __restrict__ w1,
                                              const float* __restrict__ vm) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int o = blockIdx.x % 8;
    int grp = blockIdx.x / 8;
    int slot = (grp * WAVES + wave) * 16 + (lane & 15);
    int t = -1, Pb = -1;
    if (slot < nl_count) {
        Pb = nonleaf[nl_start + slot];
        int2 ch = child[Pb];
        if ((ch.y >> o) & 1) t = ch.x + __popc(ch.y & ((1 << o) - 1));
    }
    if (!__ballot(t >= 0)) return;
    v4f acc[NP / 16];
    load_acc<NP>(acc, t >= 0 ? psi_d + size_t(t) * NP : nullptr, lane);
    if (has_l2l) gemm_f32<NP>(acc, l2l + size_t(o) * NP * NP, t >= 0 ? phi_d + size_t(Pb) * NP : nullptr, lane);
    c2e_apply<NP>(acc, w1, vm, lane);
    store_acc<NP>(acc, t >= 0 ? phi_d + size_t(t) * NP : nullptr, lane);
}

// ------------------------------------------------------------------ leaf evaluation: L2P + M2P
// Forward: (u, E) per target.  Backward: from the forward densities E and H.v
// (v = Ebar of the target), from the adjoint densities psi and E_psi.
struct FarOut {
    float* u;      // forward: float4 [N] (u, Ex, Ey, Ez) sorted
    float* b;      // backward: float [10][N] (E1 xyz, HE xyz, psi, Epsi xyz) sorted
};

template <int NP, bool BWD>
__global__ __launch_bounds__(128) void k_far(const int* __restrict__ leaves, int b2,
                                             const int4* __restrict__ anchor, const int2* __restrict__ range,
                                             const int* __restrict__ woff, const int* __restrict__ widx,
                                             const float4* __restrict__ pts, const float4* __restrict__ src2,
                                             const float* __restrict__ phi_d, const float* __restrict__ phi_u,
                                             size_t rhs_stride, const float4* __restrict__ surf, int n,
                                             BoxGeom geo, float cst, int64_t N, FarOut out) {
    __shared__ float dens[2][NP];
    __shared__ float4 sf[NP];
    const int b = leaves[blockIdx.x];
    const int4 ab = anchor[b];
    const int2 r = range[b];
    for (int t0 = r.x; t0 < r.y; t0 += blockDim.x) {
        const int i = t0 + threadIdx.x;
        const bool act = i < r.y;
        float4 x = act ? pts[i] : make_float4(0, 0, 0, 0);
        float4 eb = (BWD && act) ? src2[i] : make_float4(0, 0, 0, 0);
        // accumulators (true units without c)
        float u = 0, ex = 0, ey = 0, ez = 0;          // forward u,E  | backward E1
        float hx = 0, hy = 0, hz = 0;                 // backward H.Ebar (forward density)
        float ps = 0, px = 0, py = 0, pz = 0;         // backward psi, E_psi (adjoint density)
        int nsrc = (ab.w >= 2 && b >= b2 ? 1 : 0) + (woff[b + 1] - woff[b]);
        for (int k = 0; k < nsrc; ++k) {
            int A;
            const float4* S;
            const float* D;
            if (ab.w >= 2 && k == 0) {
                A = b;
                S = surf + NP;      // downward equivalent surface
                D = phi_d;
            } else {
                A = widx[woff[b] + k - (ab.w >= 2 ? 1 : 0)];
                S = surf;           // upward equivalent surface
                D = phi_u;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < NP; e += blockDim.x) {
                dens[0][e] = D[size_t(A) * NP + e];
                if (BWD) dens[1][e] = D[rhs_stride + size_t(A) * NP + e];
                sf[e] = S[e];
            }
            __syncthreads();
            float c[3], invw, w;
            box_frame(geo, anchor[A], c, invw, w);
            float xx = (x.x - c[0]) * invw, xy = (x.y - c[1]) * invw, xz = (x.z - c[2]) * invw;
            float su = 0, sx = 0, sy = 0, sz = 0, shx = 0, shy = 0, shz = 0, s2u = 0, s2x = 0, s2y = 0, s2z = 0;
            float vx = eb.y * invw, vy = eb.z * invw, vz = eb.w * invw;   // unused in forward
            if (act) {
                for (int e = 0; e < n; ++e) {
                    float4 s = sf[e];
                    float dx = xx - s.x, dy = xy - s.y, dz = xz - s.z;
                    float ri = rsq(dx * dx + dy * dy + dz * dz);
                    float ri3 = ri * ri * ri;
                    float f = dens[0][e];
                    if (!BWD) {
                        su += f * ri;
                        float g = f * ri3;
                        sx += g * dx;
                        sy += g * dy;
                        sz += g * dz;
                    } else {
                        float g = f * ri3;
                        sx += g * dx;
                        sy += g * dy;
                        sz += g * dz;
                        // H(r) v = 3 r (r.v) / r^5 - v / r^3   (v = Ebar in box units)
                        float ri5 = ri3 * ri * ri;
                        float rv = dx * vx + dy * vy + dz * vz;
                        float h3 = 3.f * f * rv * ri5;
                        shx += h3 * dx - g * vx;
                        shy += h3 * dy - g * vy;
                        shz += h3 * dz - g * vz;
                        float f2 = dens[1][e];
                        float g2 = f2 * ri3;
                        s2u += f2 * ri;
                        s2x += g2 * dx;
                        s2y += g2 * dy;
                        s2z += g2 * dz;
                    }
                }
            }
            float iw2 = invw * invw;
            if (!BWD) {
                u += su * invw;
                ex += sx * iw2;
                ey += sy * iw2;
                ez += sz * iw2;
            } else {
                ex += sx * iw2;
                ey += sy * iw2;
                ez += sz * iw2;
                // v was scaled by invw, so H.v picks up invw^3 / invw = invw^2 ... times invw: see below
                hx += shx * iw2;
                hy += shy * iw2;
                hz += shz * iw2;
                ps += s2u * invw;
                px += s2x * iw2;
                py += s2y * iw2;
                pz += s2z * iw2;
            }
        }
        if (act) {
            if (!BWD) {
                reinterpret_cast<float4*>(out.u)[i] = make_float4(cst * u, cst * ex, cst * ey, cst * ez);
            } else {
                float* o = out.b;
                o[0 * N + i] = cst * ex;
                o[1 * N + i] = cst * ey;
                o[2 * N + i] = cst * ez;
                o[3 * N + i] = cst * hx;
                o[4 * N + i] = cst * hy;
                o[5 * N + i] = cst * hz;
                o[6 * N + i] = cst * ps;
                o[7 * N + i] = cst * px;
                o[8 * N + i] = cst * py;
                o[9 * N + i] = cst * pz;
            }
        }
    }
}

__global__ void k_fill0(float* __restrict__ p, size_t n) {
    size_t i = blockIdx.x * size_t(256) + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

int nblk(int64_t n, int per) { return int((n + per - 1) / per); }

const VOps& vops_host() {
    static VOps v;
    static bool made = false;
    if (!made) {
        for (int o = 0; o < 8; ++o) {
            int ob[3] = {(o >> 2) & 1, (o >> 1) & 1, o & 1};
            int m = 0, j = 0;
            for (int dx = -3; dx <= 3; ++dx)
                for (int dy = -3; dy <= 3; ++dy)
                    for (int dz = -3; dz <= 3; ++dz) {
                        if (std::max(abs(dx), std::max(abs(dy), abs(dz))) <= 1) continue;
                        int d[3] = {dx, dy, dz};
                        bool ok = true;
                        for (int k = 0; k < 3; ++k) {
                            int vv = d[k] + ob[k];
                            int oo = ((vv % 2) + 2) % 2;
                            int DD = (vv - oo) / 2 + 1;
                            if (DD < 0 || DD > 2) ok = false;
                        }
                        if (ok) v.op[o][j++] = short(m);
                        ++m;
                    }
        }
        made = true;
    }
    return v;
}

template <int NP>
void sweep_impl(kifmm_plan* P, int rhs, bool dipole, hipStream_t s, bool rec) {
    const Operators& op = *P->ops;
    const int B = int(P->B);
    const size_t stride = size_t(B) * NP;
    float* psi_u = P->psi_u.as<float>() + rhs * stride;
    float* phi_u = P->phi_u.as<float>() + rhs * stride;
    float* psi_d = P->psi_d.as<float>() + rhs * stride;
    float* phi_d = P->phi_d.as<float>() + rhs * stride;
    BoxGeom geo{{P->lo[0], P->lo[1], P->lo[2]}, P->side};
    const float4* pts = P->pts.as<float4>();
    const float4* src2 = dipole ? P->src2.as<float4>() : nullptr;
    const float4* surf = op.surf.as<float4>();
    const int depth = P->depth;
    if (depth < 2) {
        if (rec) for (int k = 0; k < 5; ++k) record_phase(P, k, s);
        return;
    }
    const int b2 = int(P->lev[2].start);
    int tpb = std::min(320, (NP + 63) / 64 * 64);
    // P2M
    hipLaunchKernelGGL(k_p2m<NP>, dim3(unsigned(P->nleaves)), dim3(tpb), 0, s, P->leaves.as<int>(), int(P->nleaves),
                       b2, P->bx_anchor.as<int4>(), P->bx_range.as<int2>(), pts, src2, surf, op.n, geo, psi_u);
    if (rec) record_phase(P, 0, s);
    // upward M2M + UC2E, deepest level first
    for (int l = depth; l >= 2; --l) {
        int nb = int(P->lev[l].count);
        hipLaunchKernelGGL(k_up<NP>, dim3(nblk(nb, WAVES * 16)), dim3(WAVES * 64), 0, s, int(P->lev[l].start), nb,
                           P->bx_child.as<int2>(), P->bx_leaf.as<int>(), psi_u, phi_u, op.m2m.as<float>(),
                           op.uc2e_w1.as<float>(), op.uc2e_v.as<float>());
    }
    if (rec) record_phase(P, 1, s);
    // downward check potentials: zero, X list, V list
    size_t nz = size_t(B - b2) * NP;
    hipLaunchKernelGGL(k_fill0, dim3(unsigned((nz + 255) / 256)), dim3(256), 0, s, psi_d + size_t(b2) * NP, nz);
    if (P->n_xboxes > 0)
        hipLaunchKernelGGL(k_p2l<NP>, dim3(unsigned(P->n_xboxes)), dim3(tpb), 0, s, P->xboxes.as<int>(),
                           P->x_off.as<int>(), P->x_idx.as<int>(), P->bx_anchor.as<int4>(), P->bx_range.as<int2>(), pts,
                           src2, surf, op.n, geo, psi_d);
    if (rec) record_phase(P, 2, s);
    TaskTable tt{};
    int blocks = 0;
    for (int l = 2; l <= depth; ++l) {
        const LevelInfo& pl = P->lev[l - 1];
        int groups = nblk(pl.nl_count, WAVES * 16);
        tt.first[tt.nlev] = blocks;
        tt.level[tt.nlev] = l;
        tt.nl_start[tt.nlev] = int(pl.nl_start);
        tt.nl_count[tt.nlev] = int(pl.nl_count);
        tt.groups[tt.nlev] = groups;
        tt.nlev++;
        blocks += groups * 8;
    }
    static DBuf* vops_dev = nullptr;
    if (!vops_dev) {
        vops_dev = new DBuf();
        vops_dev->ensure(sizeof(VOps));
        KIFMM_HIP(hipMemcpy(vops_dev->p, &vops_host(), sizeof(VOps), hipMemcpyHostToDevice));
    }
    if (blocks > 0) {
        if (P->opt.precision == KIFMM_SPLIT_BF16)
            hipLaunchKernelGGL((k_m2l<NP, true>), dim3(blocks), dim3(WAVES * 64), 0, s, tt, P->nonleaf.as<int>(),
                               P->bx_child.as<int2>(), P->vdense.as<int>(), b2, vops_dev->as<VOps>(), phi_u, psi_d,
                               op.m2l.as<float>(), op.m2l_hi.as<__bf16>(), op.m2l_lo.as<__bf16>());
        else
            hipLaunchKernelGGL((k_m2l<NP, false>), dim3(blocks), dim3(WAVES * 64), 0, s, tt, P->nonleaf.as<int>(),
                               P->bx_child.as<int2>(), P->vdense.as<int>(), b2, vops_dev->as<VOps>(), phi_u, psi_d,
                               op.m2l.as<float>(), op.m2l_hi.as<__bf16>(), op.m2l_lo.as<__bf16>());
    }
    if (rec) record_phase(P, 3, s);
    for (int l = 2; l <= depth; ++l) {
        const LevelInfo& pl = P->lev[l - 1];
        int groups = nblk(pl.nl_count, WAVES * 16);
        if (groups == 0) continue;
        hipLaunchKernelGGL(k_down<NP>, dim3(groups * 8), dim3(WAVES * 64), 0, s, int(pl.nl_start), int(pl.nl_count),
                           l >= 3 ? 1 : 0, P->nonleaf.as<int>(), P->bx_child.as<int2>(), psi_d, phi_d,
                           op.l2l.as<float>(), op.dc2e_w1.as<float>(), op.dc2e_v.as<float>());
    }
    if (rec) record_phase(P, 4, s);
}

template <int NP>
void far_impl(kifmm_plan* P, bool bwd, hipStream_t s) {
    const Operators& op = *P->ops;
    BoxGeom geo{{P->lo[0], P->lo[1], P->lo[2]}, P->side};
    const int b2 = P->depth >= 2 ? int(P->lev[2].start) : int(P->B);
    FarOut fo{P->far.as<float>(), P->far.as<float>()};
    size_t stride = size_t(P->B) * NP;
    if (bwd)
        hipLaunchKernelGGL((k_far<NP, true>), dim3(unsigned(P->nleaves)), dim3(128), 0, s, P->leaves.as<int>(), b2,
                           P->bx_anchor.as<int4>(), P->bx_range.as<int2>(), P->w_off.as<int>(), P->w_idx.as<int>(),
                           P->pts.as<float4>(), P->src2.as<float4>(), P->phi_d.as<float>(), P->phi_u.as<float>(),
                           stride, op.surf.as<float4>(), op.n, geo, float(P->c), P->N, fo);
    else
        hipLaunchKernelGGL((k_far<NP, false>), dim3(unsigned(P->nleaves)), dim3(128), 0, s, P->leaves.as<int>(), b2,
                           P->bx_anchor.as<int4>(), P->bx_range.as<int2>(), P->w_off.as<int>(), P->w_idx.as<int>(),
                           P->pts.as<float4>(), (const float4*)nullptr, P->phi_d.as<float>(), P->phi_u.as<float>(),
                           stride, op.surf.as<float4>(), op.n, geo, float(P->c), P->N, fo);
}

}  // namespace

void run_sweep(kifmm_plan* P, int rhs, bool dipole, hipStream_t s, bool record) {
    switch (P->npad) {
        case 32: sweep_impl<32>(P, rhs, dipole, s, record); break;
        case 64: sweep_impl<64>(P, rhs, dipole, s, record); break;
        case 128: sweep_impl<128>(P, rhs, dipole, s, record); break;
        case 160: sweep_impl<160>(P, rhs, dipole, s, record); break;
        case 224: sweep_impl<224>(P, rhs, dipole, s, record); break;
        case 320: sweep_impl<320>(P, rhs, dipole, s, record); break;
        default: throw Error(KIFMM_ERR_ARG, "unsupported surface size");
    }
}

void run_far_eval(kifmm_plan* P, bool backward, const float*, hipStream_t s) {
    switch (P->npad) {
        case 32: far_impl<32>(P, backward, s); break;
        case 64: far_impl<64>(P, backward, s); break;
        case 128: far_impl<128>(P, backward, s); break;
        case 160: far_impl<160>(P, backward, s); break;
        case 224: far_impl<224>(P, backward, s); break;
        case 320: far_impl<320>(P, backward, s); break;
        default: throw Error(KIFMM_ERR_ARG, "unsupported surface size");
    }
}

}  // namespace kifmm
