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
#include <stdlib.h>

#include <algorithm>

#include <functional>

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

// Centre (FP64 to FP32), width and inverse width of a box; `sgn` times the
// image shift of list entry e (whole root widths) is added to the centre.
__device__ inline void box_frame(const BoxGeom& g, int4 a, float c[3], float& invw, float& w, int e = 0,
                                 int sgn = 1) {
    int sx, sy, sz;
    img_shift(e, sx, sy, sz);
    double wd = ldexp(g.side, -a.w);
    c[0] = float(g.lo[0] + (double(a.x) + 0.5) * wd + sgn * sx * g.side);
    c[1] = float(g.lo[1] + (double(a.y) + 0.5) * wd + sgn * sy * g.side);
    c[2] = float(g.lo[2] + (double(a.z) + 0.5) * wd + sgn * sz * g.side);
    w = float(wd);
    invw = float(ldexp(1.0, a.w) / g.side);
}

// c_a - c_b of two boxes of the cell (no image shift): FP64, then FP32
__device__ inline void centre_diff(const BoxGeom& g, int4 a, int4 b, float d[3]) {
    const double wa = ldexp(g.side, -a.w), wb = ldexp(g.side, -b.w);
    d[0] = float((double(a.x) + 0.5) * wa - (double(b.x) + 0.5) * wb);
    d[1] = float((double(a.y) + 0.5) * wa - (double(b.y) + 0.5) * wb);
    d[2] = float((double(a.z) + 0.5) * wa - (double(b.z) + 0.5) * wb);
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
// psi[i] = sum_j q_j K1(s_i - x'_j) - (1/w) Ebar_j . G1(s_i - x'_j)   (dipole part optional);
// with frc (the Stokeslet's fourth charge) q_j = (x_j - c) . f_j about this box's centre.
// A block has 2 NP threads: thread (slice, i) takes check point i and every
// other staged source point; the two slices are added in a fixed order.  No
// distance vanishes: the points of a leaf lie inside the upward check surface
// of their box, and an X-list leaf is separated from the downward check
// surface of its target box.
template <int NP>
__device__ void points_to_surface(float& acc, const float4* __restrict__ pts, const float4* __restrict__ src2,
                                  const float4* __restrict__ frc, int j0, int j1, const float c[3], float invw,
                                  float4 s, bool active, int slice, float4* sh, float4* sh2) {
    for (int base = j0; base < j1; base += 256) {
        const int m = min(256, j1 - base);
        __syncthreads();
        for (int k = threadIdx.x; k < m; k += blockDim.x) {
            const float4 p = pts[base + k];
            const float px = p.x - c[0], py = p.y - c[1], pz = p.z - c[2];
            float q = p.w;
            if (frc) {
                const float4 f = frc[base + k];
                q = px * f.x + py * f.y + pz * f.z;
            }
            sh[k] = make_float4(px * invw, py * invw, pz * invw, q);
            if (src2) {
                const float4 a = src2[base + k];
                sh2[k] = make_float4(a.x, a.y * invw, a.z * invw, a.w * invw);
            }
        }
        __syncthreads();
        if (active) {
            if (!src2) {
                for (int k = slice; k < m; k += 2) {
                    const float4 p = sh[k];
                    const float dx = s.x - p.x, dy = s.y - p.y, dz = s.z - p.z;
                    acc += p.w * __frsqrt_rn(dx * dx + dy * dy + dz * dz);
                }
            } else {
                for (int k = slice; k < m; k += 2) {
                    const float4 p = sh[k];
                    const float4 a = sh2[k];
                    const float dx = s.x - p.x, dy = s.y - p.y, dz = s.z - p.z;
                    const float ri = __frsqrt_rn(dx * dx + dy * dy + dz * dz);
                    const float ri3 = ri * ri * ri;
                    acc += a.x * ri - (a.y * dx + a.z * dy + a.w * dz) * ri3;
                }
            }
        }
    }
}

// slice 1 hands its partial sum to slice 0 (fixed order), which returns the total
template <int NP>
__device__ inline float add_slices(float acc, int i, int slice, float* red) {
    __syncthreads();
    if (slice == 1) red[i] = acc;
    __syncthreads();
    return slice == 0 ? acc + red[i] : 0.f;
}

template <int NP>
__global__ __launch_bounds__(2 * NP) void k_p2m(const int* __restrict__ leaves, int nleaves, int b2,
                                                const int4* __restrict__ anchor, const int2* __restrict__ range,
                                                const float4* __restrict__ pts, const float4* __restrict__ src2,
                                                const float4* __restrict__ frc, const float4* __restrict__ surf,
                                                int n, BoxGeom geo, float* __restrict__ psi_u) {
    __shared__ float4 sh[256];
    __shared__ float4 sh2[256];
    __shared__ float red[NP];
    const int b = leaves[blockIdx.x];
    if (b < b2) return;   // leaves above the first far-field level have no far field
    const int4 a = anchor[b];
    float c[3], invw, w;
    box_frame(geo, a, c, invw, w);
    const int2 r = range[b];
    const int i = threadIdx.x % NP, slice = threadIdx.x / NP;
    const bool act = i < n;
    const float4 s = act ? surf[NP + i] : make_float4(0, 0, 0, 0);   // upward check surface
    float acc = 0.f;
    points_to_surface<NP>(acc, pts, src2, frc, r.x, r.y, c, invw, s, act, slice, sh, sh2);
    acc = add_slices<NP>(acc, i, slice, red);
    if (slice == 0) psi_u[size_t(b) * NP + i] = act ? acc : 0.f;
}

template <int NP>
__global__ __launch_bounds__(2 * NP) void k_p2l(const int* __restrict__ xboxes, const int* __restrict__ xoff,
                                                const int* __restrict__ xidx, const int4* __restrict__ anchor,
                                                const int2* __restrict__ range, const float4* __restrict__ pts,
                                                const float4* __restrict__ src2, const float4* __restrict__ frc,
                                                const float4* __restrict__ surf, int n, BoxGeom geo,
                                                float* __restrict__ psi_d) {
    __shared__ float4 sh[256];
    __shared__ float4 sh2[256];
    __shared__ float red[NP];
    __builtin_amdgcn_s_setprio(2);   // issue ahead of the near-field waves sharing the SIMD
    const int b = xboxes[blockIdx.x];
    const int4 a = anchor[b];
    const int i = threadIdx.x % NP, slice = threadIdx.x / NP;
    const bool act = i < n;
    const float4 s = act ? surf[i] : make_float4(0, 0, 0, 0);   // downward check surface
    float acc = 0.f;
    for (int k = xoff[b]; k < xoff[b + 1]; ++k) {
        const int e = xidx[k];
        const int2 r = range[img_box(e)];
        // a source image shifted by +s cell widths is the target frame shifted by -s
        float c[3], invw, w;
        box_frame(geo, a, c, invw, w, e, -1);
        points_to_surface<NP>(acc, pts, src2, frc, r.x, r.y, c, invw, s, act, slice, sh, sh2);
    }
    acc = add_slices<NP>(acc, i, slice, red);
    if (slice == 0) psi_d[size_t(b) * NP + i] = act ? acc : 0.f;
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

// Hardware dispatch sends block b to XCD b % 8; give every XCD a contiguous
// range of logical tiles so that neighbouring tiles share that XCD's L2.
__device__ inline int xcd_remap(int b, int nb) {
    const int q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

typedef __attribute__((address_space(3))) void lds_void;

// Asynchronous 16-byte copy global -> LDS: lane i of the wave writes
// wave_base[i] (the LDS address is wave-uniform, the lanes are contiguous).
// Completion is tracked by vmcnt like a load.
__device__ inline void dma16(const uint4* __restrict__ g, uint4* wave_base) {
    __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)wave_base, 16, 0, 0);
}

// Copy WORDS 16-byte words of an operator chunk into LDS; word w of the chunk
// lands at dst[w] (thread tid moves words tid, tid + 256, ...).
template <int WORDS>
__device__ inline void dma_chunk(const uint4* __restrict__ g, uint4* dst, int tid) {
    const int wave = tid >> 6;
#pragma unroll
    for (int i = 0; i < (WORDS + 255) / 256; ++i)
        if (WORDS % 256 == 0 || i * 256 + wave * 64 < WORDS) dma16(g + i * 256 + tid, dst + i * 256 + wave * 64);
}

__device__ inline int next_slot(const unsigned* mk, int j) {
    for (int k = j + 1; k < kVPerOct;) {
        unsigned w = mk[k >> 5] >> (k & 31);
        if (w) return k + __builtin_ctz(w);
        k = (k | 31) + 1;
    }
    return kVPerOct;
}

__device__ inline v8bf as_bf8(uint4 u) {
    v8bf r;
    __builtin_memcpy(&r, &u, 16);
    return r;
}

__device__ inline void load8(float* b, const float* __restrict__ p) {
    if (p) {
        float4 b0 = *reinterpret_cast<const float4*>(p);
        float4 b1 = *reinterpret_cast<const float4*>(p + 4);
        b[0] = b0.x; b[1] = b0.y; b[2] = b0.z; b[3] = b0.w;
        b[4] = b1.x; b[5] = b1.y; b[6] = b1.z; b[7] = b1.w;
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) b[i] = 0.f;
    }
}

// M2L over the V lists of all levels >= 2 in one launch.  A block owns the
// targets at octant o of 4*TG*16 consecutive non-leaf parents (TG = CB/nrhs
// column blocks of 16 targets per wave, each with nrhs right-hand sides), so
// every target of the block uses the same operator in V slot j.  The block
// walks the slots that any of its targets uses; each operator is streamed in
// 32-column chunks (fragment order, NP/16*128 words) through a double-buffered
// LDS tile shared by the four waves, while the next chunk and the next source
// columns are already in flight.
// STK (a Stokes sweep, two right-hand sides: f_z, then the fourth charge in
// per-box frames): each source column of the second adds (c_source -
// c_target) times the source box's columns of f_x, f_y (s0, s1) and of f_z,
// the first right-hand side's column of the same source (s2 is not read).
template <int NP, bool SPLIT, int CB, bool STK>
__global__ __launch_bounds__(256, STK ? 2 : 3) void k_m2l(TaskTable tt, int nblk, int ntile, int nsplit, int nrhs,
                                             const int* __restrict__ nonleaf, const int2* __restrict__ child,
                                             const int* __restrict__ vdense, int b2, const VOps* __restrict__ vops,
                                             const float* __restrict__ phi_u, const float* __restrict__ psi_d,
                                             const int* __restrict__ xflag, float* __restrict__ psi_m,
                                             size_t rhs_stride, size_t split_stride, const uint4* __restrict__ ops,
                                             const int4* __restrict__ anchor, BoxGeom geo,
                                             const float* __restrict__ s0, const float* __restrict__ s1,
                                             const float* __restrict__ s2) {
    constexpr int RB = NP / 16, KC = NP / 32, WORDS = RB * 128;
    __shared__ uint4 lds0[WORDS];
    __shared__ uint4 lds1[WORDS];
    __shared__ unsigned vmask[6];
    __shared__ short sop[kVPerOct];   // operator index of each V slot of octant o
    __builtin_amdgcn_s_setprio(2);   // issue ahead of the near-field waves sharing the SIMD
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, tid = threadIdx.x;
    // logical tile order (split, level, parent group, octant): the blocks an
    // XCD runs together are the eight octants of neighbouring parent groups,
    // which read the same source boxes (the children of the parents'
    // colleagues) through one slot range; this reuse of sources in L2 paid
    // more than the octant-major order's reuse of operators
    const int lid = xcd_remap(blockIdx.x, nblk);
    const int split = lid / ntile, rest = lid % ntile;
    const int o = rest % 8, bid = rest / 8;
    const int j_lo = split * kVPerOct / nsplit, j_hi = (split + 1) * kVPerOct / nsplit;
    int e = 0;
    while (e + 1 < tt.nlev && bid >= tt.first[e + 1]) ++e;
    const int grp = bid - tt.first[e];
    const int TG = CB / nrhs;
    int tgt[CB];
    const float* bsrc[CB];
    const int* vrow[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int tg = cb / nrhs;
        const int slot = ((grp * WAVES + wave) * TG + tg) * 16 + (lane & 15);
        int t = -1;
        if (slot < tt.nl_count[e]) {
            const int2 ch = child[nonleaf[tt.nl_start[e] + slot]];
            if ((ch.y >> o) & 1) t = ch.x + __popc(ch.y & ((1 << o) - 1));
        }
        tgt[cb] = t;
        vrow[cb] = t >= 0 ? vdense + size_t(t - b2) * kVPerOct : nullptr;
        bsrc[cb] = phi_u + size_t(cb % nrhs) * rhs_stride;
    }
    if (tid < 6) vmask[tid] = 0;
    for (int k = tid; k < kVPerOct; k += 256) sop[k] = vops->op[o][k];
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 6; ++w) {
        unsigned m = 0;
        const int lo = max(j_lo, 32 * w), hi = min(j_hi, 32 * w + 32);
        for (int cb = 0; cb < CB; cb += nrhs)
            if (vrow[cb])
                for (int jj = lo; jj < hi; ++jj)
                    if (vrow[cb][jj] >= 0) m |= 1u << (jj & 31);
        if (m) atomicOr(&vmask[w], m);
    }
    __syncthreads();
    int j = next_slot(vmask, -1);   // block-uniform; kVPerOct when this slot range is empty
    // split 0 of a target that the P2L kernel wrote starts from its X-list
    // check potential (no other box's value is written before), the others
    // from zero
    v4f acc[CB][RB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
        load_acc<NP>(acc[cb],
                     (split == 0 && tgt[cb] >= 0 && psi_d && xflag[tgt[cb]])
                         ? psi_d + size_t(cb % nrhs) * rhs_stride + size_t(tgt[cb]) * NP
                         : nullptr,
                     lane);
    if (j < kVPerOct) {
        const int g8 = 8 * (lane >> 4);
        int kc = 0;
        float breg[CB][8];
        const float* col[CB];
        // STK: the source box of each column at the current slot, its shift
        // into the target's frame, and its f_x, f_y columns (odd columns)
        int sidx[CB];
        float dsh[CB][3];
        float bxr[CB][8], byr[CB][8];
        // source index of each column at the slot after the current one, read
        // one slot ahead so that a slot change never waits for it
        int pre[CB];
        auto read_pre = [&](int jj) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) pre[cb] = (vrow[cb] && jj < kVPerOct) ? vrow[cb][jj] : -1;
        };
        // start chunk (jj, kk): operator words by DMA into dst, source columns into breg
        auto issue = [&](int jj, int kk, bool newslot, uint4* dst) {
            if (newslot) {
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    col[cb] = pre[cb] >= 0 ? bsrc[cb] + size_t(pre[cb]) * NP : nullptr;
                    if constexpr (STK) {
                        sidx[cb] = pre[cb];
                        dsh[cb][0] = dsh[cb][1] = dsh[cb][2] = 0.f;
                        if ((cb & 1) && pre[cb] >= 0) centre_diff(geo, anchor[pre[cb]], anchor[tgt[cb]], dsh[cb]);
                    }
                }
            }
            dma_chunk<WORDS>(ops + (size_t(sop[jj]) * KC + kk) * WORDS, dst, tid);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) load8(breg[cb], col[cb] ? col[cb] + kk * 32 + g8 : nullptr);
            if constexpr (STK) {
#pragma unroll
                for (int cb = 1; cb < CB; cb += 2) {
                    const size_t o8 = size_t(sidx[cb] >= 0 ? sidx[cb] : 0) * NP + kk * 32 + g8;
                    load8(bxr[cb], sidx[cb] >= 0 ? s0 + o8 : nullptr);
                    load8(byr[cb], sidx[cb] >= 0 ? s1 + o8 : nullptr);
                }
            }
            if (newslot) read_pre(next_slot(vmask, jj));
        };
        // one chunk: wait until it has landed (all waves), start the next one
        // into the other buffer, multiply
        auto step = [&](const uint4* L, uint4* other) -> bool {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            float cur[CB][8];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    cur[cb][i] = breg[cb][i];
                    if constexpr (STK)
                        if (cb & 1)
                            cur[cb][i] += dsh[cb][0] * bxr[cb][i] + dsh[cb][1] * byr[cb][i] +
                                          dsh[cb][2] * breg[cb - 1][i];
                }
            int nkc = kc + 1, nj = j;
            if (nkc == KC) {
                nkc = 0;
                nj = next_slot(vmask, j);
            }
            if (nj < kVPerOct) issue(nj, nkc, nj != j, other);
            if (SPLIT) {
                v8bf bh[CB], bl[CB];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        __bf16 h = (__bf16)cur[cb][i];
                        bh[cb][i] = h;
                        bl[cb][i] = (__bf16)(cur[cb][i] - (float)h);
                    }
                // the fragments of row block rb + 1 are read while rb multiplies
                uint4 nh = L[lane], nl = L[64 + lane];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const v8bf ah = as_bf8(nh);
                    const v8bf al = as_bf8(nl);
                    if (rb + 1 < RB) {
                        nh = L[(rb + 1) * 128 + lane];
                        nl = L[(rb + 1) * 128 + 64 + lane];
                    }
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        v4f c = acc[cb][rb];
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[cb], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[cb], c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[cb], c, 0, 0, 0);
                        acc[cb][rb] = c;
                    }
                }
            } else {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const uint4 u0 = L[rb * 128 + lane];
                    const uint4 u1 = L[rb * 128 + 64 + lane];
                    const float a[8] = {__uint_as_float(u0.x), __uint_as_float(u0.y), __uint_as_float(u0.z),
                                        __uint_as_float(u0.w), __uint_as_float(u1.x), __uint_as_float(u1.y),
                                        __uint_as_float(u1.z), __uint_as_float(u1.w)};
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        v4f c = acc[cb][rb];
#pragma unroll
                        for (int i = 0; i < 8; ++i)
                            c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], cur[cb][i], c, 0, 0, 0);
                        acc[cb][rb] = c;
                    }
                }
            }
            j = nj;
            kc = nkc;
            return j < kVPerOct;
        };
        read_pre(j);
        issue(j, 0, true, lds0);
        // the two buffers alternate in a fixed order, so every LDS read names one buffer
        while (step(lds0, lds1) && step(lds1, lds0)) {
        }
    }
    float* out = psi_m + size_t(split) * split_stride;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
        store_acc<NP>(acc[cb], tgt[cb] >= 0 ? out + size_t(cb % nrhs) * rhs_stride + size_t(tgt[cb]) * NP : nullptr,
                      lane);
}

// ------------------------------------------------------------------ upward and downward translations
// Upward (UP): for the boxes list[b0 .. b0+nb) (the leaves of every level, or
// the non-leaves of one), psi = P2M result (leaves) or sum_o M2M[o]
// phi_u(child o) (non-leaves), then phi_u = V (W1 psi).
// Downward: for the children at octant o of non-leaf parents, psi = the summed
// M2L partials (+ X list) + L2L[o] phi_d(parent) (from level 3), then
// phi_d = U (W1d psi).
// A block holds 16 boxes (one MFMA column block) and its four waves split the
// NP/16 output row blocks (wave w owns rb = w, w + 4, ...), so that even a
// level with a few boxes is spread over several SIMDs.  The operators (under
// 1 MB) are read as MFMA fragments straight from L2.  The chained
// check-to-equivalent factors need the whole intermediate vector: it is
// exchanged through LDS in accumulator layout.
// STK (the Stokeslet's fourth charge in per-box frames): every gathered
// source column adds (c_source - c_target) times the same box's densities of
// the three force components (s0, s1, s2), which moves it into the target's
// frame.
template <int NP, bool UP, bool STK>
__global__ __launch_bounds__(256) void k_updown(int nblk, int b0, int nb, const int* __restrict__ list, int nl_start,
                                                int nl_count, int has_l2l,
                                                const int* __restrict__ nonleaf, const int2* __restrict__ child,
                                                const int* __restrict__ leafflag, const float* __restrict__ psi_in,
                                                int nsplit, size_t split_stride, const float* __restrict__ gsrc,
                                                float* __restrict__ out, const uint4* __restrict__ gops,
                                                const uint4* __restrict__ w1c, const uint4* __restrict__ vc,
                                                const int4* __restrict__ anchor, BoxGeom geo,
                                                const float* __restrict__ s0, const float* __restrict__ s1,
                                                const float* __restrict__ s2) {
    constexpr int RB = NP / 16, KC = NP / 32, NR = (RB + 3) / 4;
    __shared__ v4f xa[RB][64];
    __builtin_amdgcn_s_setprio(2);   // issue ahead of the near-field waves sharing the SIMD
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int bid = xcd_remap(blockIdx.x, nblk);
    const int g4 = 4 * (lane >> 4), g8 = 8 * (lane >> 4);
    int tgt = -1, par = -1, cmask = 0, cfirst = 0, o = 0;
    if (UP) {
        const int idx = bid * 16 + (lane & 15);
        if (idx < nb) {
            tgt = list[b0 + idx];
            if (!leafflag[tgt]) {
                const int2 ch = child[tgt];
                cfirst = ch.x;
                cmask = ch.y;
            }
        }
    } else {
        o = bid % 8;
        const int slot = (bid / 8) * 16 + (lane & 15);
        if (slot < nl_count) {
            const int Pb = nonleaf[nl_start + slot];
            const int2 ch = child[Pb];
            if ((ch.y >> o) & 1) {
                tgt = ch.x + __popc(ch.y & ((1 << o) - 1));
                par = Pb;
            }
        }
    }
    // the gather terms any column of the block needs (every wave holds the
    // same 16 columns, so this is uniform over the block)
    int flags = 0;
    if (UP) {
#pragma unroll
        for (int oc = 0; oc < 8; ++oc)
            if (__ballot((cmask >> oc) & 1)) flags |= 1 << oc;
    } else {
        flags = __ballot(tgt >= 0) ? 1 : 0;
        if (!flags) return;
    }
    const float* col0 = tgt >= 0 ? psi_in + size_t(tgt) * NP : nullptr;
    v4f acc[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int rb = wave + 4 * i;
        acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
        if (rb < RB && col0 && !(UP && cmask)) {
            for (int sp = 0; sp < (UP ? 1 : nsplit); ++sp) {
                const float4 v = *reinterpret_cast<const float4*>(col0 + sp * split_stride + rb * 16 + g4);
                acc[i] += v4f{v.x, v.y, v.z, v.w};
            }
        }
    }
    // gather: acc += T[op] src (T in fragment order [kc][rb][2][64]); the
    // steps (term, 32-column chunk) run with the next step's fragments and
    // source values already in flight
    const int nterm = UP ? __popc(flags) : (has_l2l ? 1 : 0);
    const int nst = nterm * KC;
    auto step_src = [&](int st, const uint4*& A, const float*& b, int& sb) {
        const int t = st / KC, kc = st % KC;
        int op = o;
        if (UP) {
            int f = flags;
            for (int k = 0; k < t; ++k) f &= f - 1;
            op = __builtin_ctz(f);
        }
        sb = -1;
        if (UP) {
            if ((cmask >> op) & 1) sb = cfirst + __popc(cmask & ((1 << op) - 1));
        } else if (par >= 0) {
            sb = par;
        }
        A = gops + (size_t(op) * KC + kc) * RB * 128 + lane;
        b = sb >= 0 ? gsrc + size_t(sb) * NP + kc * 32 + g8 : nullptr;
    };
    uint4 an[NR][2];
    float bn[8];
    auto fetch = [&](int st) {
        const uint4* A;
        const float* b;
        int sb;
        step_src(st, A, b, sb);
        load8(bn, b);
        if constexpr (STK) {
            if (sb >= 0) {
                const size_t o8 = size_t(sb) * NP + (st % KC) * 32 + g8;
                float bx[8], by[8], bz[8], d[3];
                load8(bx, s0 + o8);
                load8(by, s1 + o8);
                load8(bz, s2 + o8);
                centre_diff(geo, anchor[sb], anchor[tgt], d);
#pragma unroll
                for (int k = 0; k < 8; ++k) bn[k] += d[0] * bx[k] + d[1] * by[k] + d[2] * bz[k];
            }
        }
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int rb = wave + 4 * i;
            if (rb < RB) {
                an[i][0] = A[rb * 128];
                an[i][1] = A[rb * 128 + 64];
            }
        }
    };
    if (nst > 0) fetch(0);
    for (int st = 0; st < nst; ++st) {
        uint4 ac[NR][2];
        float bc[8];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            ac[i][0] = an[i][0];
            ac[i][1] = an[i][1];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) bc[k] = bn[k];
        if (st + 1 < nst) fetch(st + 1);
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            if (wave + 4 * i < RB) {
                const float a[8] = {__uint_as_float(ac[i][0].x), __uint_as_float(ac[i][0].y),
                                    __uint_as_float(ac[i][0].z), __uint_as_float(ac[i][0].w),
                                    __uint_as_float(ac[i][1].x), __uint_as_float(ac[i][1].y),
                                    __uint_as_float(ac[i][1].z), __uint_as_float(ac[i][1].w)};
                v4f c = acc[i];
#pragma unroll
                for (int k = 0; k < 8; ++k) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k], bc[k], c, 0, 0, 0);
                acc[i] = c;
            }
        }
    }
    // chained factors: acc = V (W1 acc), the right factor read from LDS
    auto chain = [&](const uint4* __restrict__ C) {
#pragma unroll
        for (int i = 0; i < NR; ++i)
            if (wave + 4 * i < RB) xa[wave + 4 * i][lane] = acc[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int ob = wave + 4 * i;
            if (ob < RB) {
                v4f cc = v4f{0.f, 0.f, 0.f, 0.f};
                const uint4* Cr = C + size_t(ob) * RB * 64 + lane;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const uint4 u = Cr[rb * 64];
                    const v4f T = xa[rb][lane];
                    cc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(u.x), T[0], cc, 0, 0, 0);
                    cc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(u.y), T[1], cc, 0, 0, 0);
                    cc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(u.z), T[2], cc, 0, 0, 0);
                    cc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(u.w), T[3], cc, 0, 0, 0);
                }
                acc[i] = cc;
            }
        }
        __syncthreads();
    };
    chain(w1c);
    chain(vc);
    if (tgt >= 0) {
        float* dst = out + size_t(tgt) * NP;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int rb = wave + 4 * i;
            if (rb < RB)
                *reinterpret_cast<float4*>(dst + rb * 16 + g4) = make_float4(acc[i][0], acc[i][1], acc[i][2], acc[i][3]);
        }
    }
}

// ------------------------------------------------------------------ leaf evaluation: L2P + M2P
// Forward: (u, E) per target.  Backward: the far part of the adjoint
// combination xbar = -ubar E - H Ebar - q E_psi and of qbar = psi, from the
// forward (E, H) and adjoint (psi, E_psi) equivalent densities.
// Small items give each target S lanes of a wave (as in the near field) that
// split the surface points and are summed by shuffles.
struct FarOut {
    const float4* nearv;   // sorted near-field part: forward (u, E), backward (xbar, psi); or null
    const int* perm;       // sorted position -> caller index; null: outputs in sorted order
    float* a;              // forward: potential [N] | backward: grad_charges [N] (either may be null)
    float* b;              // forward: field [N][3]  | backward: grad_positions [N][3]
    // periodic: source moments (Q, M, S2, D, D.y) about the cell centre o of
    // the evaluated right-hand side (backward: the forward charges, then the
    // adjoint sources 16 doubles further), null in free space; k1 = 2 pi c / (3 V)
    const double* mom;
    double o[3];
    double k1;
    int acc;               // 1: outputs are added to instead of overwritten
    // the Stokeslet's fourth charge in per-box frames: upward densities of the
    // three force components, whose (c_A - c_leaf) multiples move a W-list
    // density into the target leaf's frame (null otherwise)
    const float* wsh[3];
};

// The non-harmonic part k1 |x - y|^2 of the periodic kernel summed over the
// sources in closed form, at y (relative to the cell centre): potential and
// field of monopoles s_j and dipoles m_j with moments
//   Q = sum s, M = sum s y, S2 = sum s |y|^2, D = sum m, DY = sum m . y.
__device__ inline void moment_terms(const double* m, double k1, const double y[3], double& u, double E[3]) {
    const double Q = m[0], S2 = m[4], DY = m[8];
    const double yy = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    const double ym = y[0] * m[1] + y[1] * m[2] + y[2] * m[3];
    const double yd = y[0] * m[5] + y[1] * m[6] + y[2] * m[7];
    u = k1 * (Q * yy - 2.0 * ym + S2 + 2.0 * yd - 2.0 * DY);
    for (int d = 0; d < 3; ++d) E[d] = 2.0 * k1 * (m[1 + d] - m[5 + d] - Q * y[d]);
}

__device__ inline int far_lanes(int nt) { return nt <= 8 ? 8 : nt <= 16 ? 4 : nt <= 32 ? 2 : 1; }

__device__ inline float far_sum(float v, int S) {
    for (int off = 1; off < S; off <<= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Work item = (leaf, first target), up to 64 targets, launched heaviest first.
// The sources are the leaf's own downward density (from the first far-field
// level) and its W-list upward densities (at their image positions).  Each source is staged in LDS as (surface point,
// density) in box units, padded to NP entries with zero density at a real
// surface point; its NP entries are dealt to the four waves and to the S
// lanes of a target inside a wave (4 S slices, static trip count).  No
// distance vanishes: the targets are inside the leaf, the downward surface
// lies outside it and a W-list box is separated from the leaf by at least its
// own width.  Wave partial sums are added in a fixed order.
template <int NP, bool BWD, int S>
__device__ __forceinline__ void far_item(int b, int first, int nt, int b2, const int4* __restrict__ anchor,
                                         const int* __restrict__ woff, const int* __restrict__ widx,
                                         const float4* __restrict__ pts, const float4* __restrict__ src2,
                                         const float* __restrict__ phi_d, const float* __restrict__ phi_u,
                                         size_t rhs_stride, const float4* __restrict__ surf, int n,
                                         const BoxGeom& geo, float cst, int64_t N, FarOut out, float4* stage,
                                         float* stage2, float* red) {
    constexpr int NV = 4, NSL = 4 * S, ITER = NP / NSL;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, tid = threadIdx.x;
    const int slice = lane & (S - 1);
    const int i = first + lane / S;
    const bool act = lane / S < nt;
    const float4 x = act ? pts[i] : make_float4(0, 0, 0, 0);
    const float4 eb = (BWD && act) ? src2[i] : make_float4(0, 0, 0, 0);
    const int self = b >= b2 ? 1 : 0;
    const int nsrc = self + (woff[b + 1] - woff[b]);
    const int sl = w * S + slice;
    // forward: (u, E) | backward: (xbar, psi) of the adjoint combination
    float v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.f;
    for (int k = 0; k < nsrc; ++k) {
        const bool own = self && k == 0;
        const int e = own ? b : widx[woff[b] + k - self];
        const int A = img_box(e);
        const float* D = (own ? phi_d : phi_u) + size_t(A) * NP;
        const float4* SF = own ? surf + NP : surf;   // downward (2.95) or upward (1.05) equivalent surface
        float dsh[3] = {0.f, 0.f, 0.f};
        const bool shift = !own && out.wsh[0];
        if (shift) centre_diff(geo, anchor[A], anchor[b], dsh);
        __syncthreads();   // the previous source is no longer read
        for (int t = tid; t < NP; t += 256) {
            const bool real = t < n;
            const float4 sp = SF[real ? t : 0];
            float dv = real ? D[t] : 0.f;
            if (shift && real) {
                const size_t at = size_t(A) * NP + t;
                dv += dsh[0] * out.wsh[0][at] + dsh[1] * out.wsh[1][at] + dsh[2] * out.wsh[2][at];
            }
            stage[t] = make_float4(sp.x, sp.y, sp.z, dv);
            if (BWD) stage2[t] = real ? D[rhs_stride + t] : 0.f;
        }
        __syncthreads();
        float c[3], invw, wd;
        box_frame(geo, anchor[A], c, invw, wd, e);
        const float xx = (x.x - c[0]) * invw, xy = (x.y - c[1]) * invw, xz = (x.z - c[2]) * invw;
        const float vx = eb.y * invw, vy = eb.z * invw, vz = eb.w * invw;   // Ebar in box units
        const float uk = eb.x, qk = x.w;
        // forward: su, (sx, sy, sz) = potential and field sums.  Backward, with
        // f1 the forward and f2 the adjoint density: xbar = -ubar_k E1 - H Ebar_k
        // - q_k E_psi summed as r [-(ubar_k f1 + q_k f2)/r^3 - 3 f1 (r.v)/r^5]
        // + (f1/r^3) v, v = Ebar_k / w; psi = sum f2/r.
        float su = 0, sx = 0, sy = 0, sz = 0, ss = 0;
#pragma unroll
        for (int m = 0; m < ITER; ++m) {
            const int e = sl + NSL * m;
            const float4 sp = stage[e];
            const float dx = xx - sp.x, dy = xy - sp.y, dz = xz - sp.z;
            const float ri = __frsqrt_rn(dx * dx + dy * dy + dz * dz);
            const float f = sp.w;
            const float ri2 = ri * ri;
            if (!BWD) {
                const float fr = f * ri;
                const float g = fr * ri2;
                su += fr;
                sx += g * dx;
                sy += g * dy;
                sz += g * dz;
            } else {
                const float f2 = stage2[e];
                const float ri3 = ri2 * ri;
                const float rv = dx * vx + dy * vy + dz * vz;
                const float coef = -ri3 * (uk * f + qk * f2) - 3.f * f * rv * ri3 * ri2;
                sx += coef * dx;
                sy += coef * dy;
                sz += coef * dz;
                ss += f * ri3;
                su += f2 * ri;
            }
        }
        // true units: potential c/w, field and position gradient c/w^2
        const float iw2 = invw * invw;
        if (!BWD) {
            v[0] += su * invw;
            v[1] += sx * iw2;
            v[2] += sy * iw2;
            v[3] += sz * iw2;
        } else {
            v[0] += (sx + ss * vx) * iw2;
            v[1] += (sy + ss * vy) * iw2;
            v[2] += (sz + ss * vz) * iw2;
            v[3] += su * invw;
        }
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = far_sum(v[q], S);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) red[(w * NV + q) * 64 + lane] = v[q];
    __syncthreads();
    if (w == 0 && act && slice == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
            v[q] = cst * (((red[q * 64 + lane] + red[(NV + q) * 64 + lane]) + red[(2 * NV + q) * 64 + lane]) +
                          red[(3 * NV + q) * 64 + lane]);
        if (out.mom) {
            // periodic: the moment terms, added to the far part in FP64
            const double y[3] = {double(x.x) - out.o[0], double(x.y) - out.o[1], double(x.z) - out.o[2]};
            double u0, E0[3];
            moment_terms(out.mom, out.k1, y, u0, E0);
            if (!BWD) {
                v[0] = float(double(v[0]) + u0);
                for (int d = 0; d < 3; ++d) v[1 + d] = float(double(v[1 + d]) + E0[d]);
            } else {
                // xbar -= ubar E + H Ebar + q E_psi with H = 2 k1 Q I; qbar += psi
                double u1, E1[3];
                moment_terms(out.mom + 16, out.k1, y, u1, E1);
                const double eb3[3] = {eb.y, eb.z, eb.w};
                for (int d = 0; d < 3; ++d)
                    v[d] = float(double(v[d]) - double(eb.x) * E0[d] - 2.0 * out.k1 * out.mom[0] * eb3[d] -
                                 double(x.w) * E1[d]);
                v[3] = float(double(v[3]) + u1);
            }
        }
        // far + near, written in caller order (sorted order without perm)
        const float4 nr = out.nearv ? out.nearv[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        const size_t j = out.perm ? size_t(out.perm[i]) : size_t(i);
        float oa, ob[3];
        if (!BWD) {
            oa = v[0] + nr.x;
            ob[0] = v[1] + nr.y;
            ob[1] = v[2] + nr.z;
            ob[2] = v[3] + nr.w;
        } else {
            oa = v[3] + nr.w;
            ob[0] = v[0] + nr.x;
            ob[1] = v[1] + nr.y;
            ob[2] = v[2] + nr.z;
        }
        if (out.a) out.a[j] = out.acc ? out.a[j] + oa : oa;
        if (out.b)
#pragma unroll
            for (int d = 0; d < 3; ++d) out.b[3 * j + d] = out.acc ? out.b[3 * j + d] + ob[d] : ob[d];
    }
}

template <int NP, bool BWD>
__global__ __launch_bounds__(256) void k_far(const int2* __restrict__ items, int b2,
                                             const int4* __restrict__ anchor, const int2* __restrict__ range,
                                             const int* __restrict__ woff, const int* __restrict__ widx,
                                             const float4* __restrict__ pts, const float4* __restrict__ src2,
                                             const float* __restrict__ phi_d, const float* __restrict__ phi_u,
                                             size_t rhs_stride, const float4* __restrict__ surf, int n,
                                             BoxGeom geo, float cst, int64_t N, FarOut out) {
    constexpr int NV = 4;
    __shared__ float red[4 * NV * 64];
    __shared__ float4 stage[NP];
    __shared__ float stage2[BWD ? NP : 1];
    const int2 it = items[blockIdx.x];
    const int b = it.x;
    const int nt = min(64, range[b].y - it.y);
#define KIFMM_FAR_ITEM(SV)                                                                                        \
    far_item<NP, BWD, SV>(b, it.y, nt, b2, anchor, woff, widx, pts, src2, phi_d, phi_u, rhs_stride, surf, n, geo, \
                          cst, N, out, stage, stage2, red)
    switch (far_lanes(nt)) {
    case 8: KIFMM_FAR_ITEM(8); break;
    case 4: KIFMM_FAR_ITEM(4); break;
    case 2: KIFMM_FAR_ITEM(2); break;
    default: KIFMM_FAR_ITEM(1); break;
    }
#undef KIFMM_FAR_ITEM
}

// Periodic moments of one right-hand side (sources s = pts.w, or with `src2`
// monopoles src2.x and dipoles src2.yzw) about the cell centre o, in FP64:
// per-block partials in a fixed order, then one block sums the partials.
__global__ __launch_bounds__(256) void k_moments(int64_t N, const float4* __restrict__ pts,
                                                 const float4* __restrict__ src2, double ox, double oy, double oz,
                                                 double* __restrict__ part) {
    __shared__ double red[9][256];
    double a[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < N; i += int64_t(gridDim.x) * 256) {
        const float4 p = pts[i];
        const double y[3] = {double(p.x) - ox, double(p.y) - oy, double(p.z) - oz};
        double sj = p.w, m[3] = {0, 0, 0};
        if (src2) {
            const float4 t = src2[i];
            sj = t.x;
            m[0] = t.y;
            m[1] = t.z;
            m[2] = t.w;
        }
        a[0] += sj;
        for (int d = 0; d < 3; ++d) a[1 + d] += sj * y[d];
        a[4] += sj * (y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
        for (int d = 0; d < 3; ++d) a[5 + d] += m[d];
        a[8] += m[0] * y[0] + m[1] * y[1] + m[2] * y[2];
    }
    for (int q = 0; q < 9; ++q) red[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (threadIdx.x < h)
            for (int q = 0; q < 9; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 9) part[size_t(blockIdx.x) * 16 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_moments_sum(const double* __restrict__ part, int nb, double* __restrict__ mom) {
    const int q = threadIdx.x;
    if (q >= 16) return;
    double t = 0.0;
    if (q < 9)
        for (int b = 0; b < nb; ++b) t += part[size_t(b) * 16 + q];
    mom[q] = t;
}

// Periodic root: downward equivalent density from the root upward density,
// phi_d = R phi_u with R = DC2E F (FP64 [n][n]); padded entries are zero.
__global__ void k_lattice(const double* __restrict__ R, int n, int np, const float* __restrict__ phi_u,
                          float* __restrict__ phi_d) {
    const int i = threadIdx.x;
    if (i >= np) return;
    double acc = 0.0;
    if (i < n)
        for (int j = 0; j < n; ++j) acc += R[size_t(i) * n + j] * double(phi_u[j]);
    phi_d[i] = float(acc);
}

// Leaf evaluation with the field gradient: (u, E, dE/dx) from the leaf's own
// downward density and its W-list upward densities (monopole densities only),
// dE_a/dx_b = sum f (delta_ab / r^3 - 3 r_a r_b / r^5), plus the near part
// (nearv, nearg) and, periodic, the moment terms (dE/dx = -2 k1 Q I).  One
// item per block, four waves over the surface points and S lanes per target.
template <int NP, int S>
__device__ __forceinline__ void far_grad_item(int b, int first, int nt, int b2, const int4* __restrict__ anchor,
                                              const int* __restrict__ woff, const int* __restrict__ widx,
                                              const float4* __restrict__ pts, const float* __restrict__ phi_d,
                                              const float* __restrict__ phi_u, const float4* __restrict__ surf,
                                              int n, const BoxGeom& geo, float cst, FarOut out,
                                              const float* __restrict__ nearg, float* __restrict__ grad,
                                              float4* stage, float* red) {
    constexpr int NV = 10, NSL = 4 * S, ITER = NP / NSL;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, tid = threadIdx.x;
    const int slice = lane & (S - 1);
    const int i = first + lane / S;
    const bool act = lane / S < nt;
    const float4 x = act ? pts[i] : make_float4(0, 0, 0, 0);
    const int self = b >= b2 ? 1 : 0;
    const int nsrc = self + (woff[b + 1] - woff[b]);
    const int sl = w * S + slice;
    float v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.f;
    for (int k = 0; k < nsrc; ++k) {
        const bool own = self && k == 0;
        const int e = own ? b : widx[woff[b] + k - self];
        const int A = img_box(e);
        const float* D = (own ? phi_d : phi_u) + size_t(A) * NP;
        const float4* SF = own ? surf + NP : surf;
        __syncthreads();
        for (int t = tid; t < NP; t += 256) {
            const bool real = t < n;
            const float4 sp = SF[real ? t : 0];
            stage[t] = make_float4(sp.x, sp.y, sp.z, real ? D[t] : 0.f);
        }
        __syncthreads();
        float c[3], invw, wd;
        box_frame(geo, anchor[A], c, invw, wd, e);
        const float xx = (x.x - c[0]) * invw, xy = (x.y - c[1]) * invw, xz = (x.z - c[2]) * invw;
        float a[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) a[q] = 0.f;
#pragma unroll
        for (int m = 0; m < ITER; ++m) {
            const float4 sp = stage[sl + NSL * m];
            const float dx = xx - sp.x, dy = xy - sp.y, dz = xz - sp.z;
            const float ri = __frsqrt_rn(dx * dx + dy * dy + dz * dz);
            const float ri2 = ri * ri;
            const float fr = sp.w * ri;
            const float g = fr * ri2;
            const float h = 3.f * g * ri2;
            a[0] += fr;
            a[1] += g * dx;
            a[2] += g * dy;
            a[3] += g * dz;
            a[4] += g - h * dx * dx;
            a[5] += g - h * dy * dy;
            a[6] += g - h * dz * dz;
            a[7] -= h * dx * dy;
            a[8] -= h * dx * dz;
            a[9] -= h * dy * dz;
        }
        // true units: potential 1/w, field 1/w^2, gradient 1/w^3
        const float iw2 = invw * invw, iw3 = iw2 * invw;
        v[0] += a[0] * invw;
#pragma unroll
        for (int q = 1; q < 4; ++q) v[q] += a[q] * iw2;
#pragma unroll
        for (int q = 4; q < NV; ++q) v[q] += a[q] * iw3;
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = far_sum(v[q], S);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) red[(w * NV + q) * 64 + lane] = v[q];
    __syncthreads();
    if (w == 0 && act && slice == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
            v[q] = cst * (((red[q * 64 + lane] + red[(NV + q) * 64 + lane]) + red[(2 * NV + q) * 64 + lane]) +
                          red[(3 * NV + q) * 64 + lane]);
        if (out.mom) {
            const double y[3] = {double(x.x) - out.o[0], double(x.y) - out.o[1], double(x.z) - out.o[2]};
            double u0, E0[3];
            moment_terms(out.mom, out.k1, y, u0, E0);
            v[0] = float(double(v[0]) + u0);
            for (int d = 0; d < 3; ++d) {
                v[1 + d] = float(double(v[1 + d]) + E0[d]);
                v[4 + d] = float(double(v[4 + d]) - 2.0 * out.k1 * out.mom[0]);
            }
        }
        const float4 nr = out.nearv[i];
        const size_t j = size_t(out.perm[i]);
        if (out.a) out.a[j] = v[0] + nr.x;
        if (out.b) {
            out.b[3 * j] = v[1] + nr.y;
            out.b[3 * j + 1] = v[2] + nr.z;
            out.b[3 * j + 2] = v[3] + nr.w;
        }
        if (grad)
            for (int q = 0; q < 6; ++q) grad[6 * j + q] = v[4 + q] + nearg[6 * size_t(i) + q];
    }
}

template <int NP>
__global__ __launch_bounds__(256) void k_far_grad(const int2* __restrict__ items, int b2,
                                                  const int4* __restrict__ anchor, const int2* __restrict__ range,
                                                  const int* __restrict__ woff, const int* __restrict__ widx,
                                                  const float4* __restrict__ pts, const float* __restrict__ phi_d,
                                                  const float* __restrict__ phi_u, const float4* __restrict__ surf,
                                                  int n, BoxGeom geo, float cst, FarOut out,
                                                  const float* __restrict__ nearg, float* __restrict__ grad) {
    __shared__ float red[4 * 10 * 64];
    __shared__ float4 stage[NP];
    const int2 it = items[blockIdx.x];
    const int b = it.x;
    const int nt = min(64, range[b].y - it.y);
#define KIFMM_FARG_ITEM(SV)                                                                                      \
    far_grad_item<NP, SV>(b, it.y, nt, b2, anchor, woff, widx, pts, phi_d, phi_u, surf, n, geo, cst, out, nearg, \
                          grad, stage, red)
    switch (far_lanes(nt)) {
    case 8: KIFMM_FARG_ITEM(8); break;
    case 4: KIFMM_FARG_ITEM(4); break;
    case 2: KIFMM_FARG_ITEM(2); break;
    default: KIFMM_FARG_ITEM(1); break;
    }
#undef KIFMM_FARG_ITEM
}

// Compressed M2L change of basis on MFMA, for the boxes [b0, b0 + nb):
//   out[b][j] = sum_k in[b][k] W[j][k]        (ACCUM: out[b][j] += ...)
// with W row-major [NOUT][NIN] and `in` the sum of nsplit arrays split_stride
// apart.  The projection phi_k = Q^T phi_u takes W = Q^T ([kp][NP]); the
// expansion psi_d += Q (sum of the partial psi_k) takes W = Q ([NP][kp]),
// adding only to the boxes whose check potentials the P2L kernel wrote
// (xflag); the others are stored.
// A wave owns 16 boxes and CPW of the NOUT/16 column tiles (v_mfma_f32_16x16x4_f32,
// operand layout as in the file header).  In a 16-wide k chunk the lane in
// group kk = lane/16 loads the float4 k0 + 4 kk .. k0 + 4 kk + 3 of its box row
// and of the W row of its column, and step s of the four MFMAs takes component
// s: k = k0 + 4 kk + s, the same permutation on both operands.
template <int NIN, int NOUT, bool ACCUM>
__global__ __launch_bounds__(256) void k_basis(int b0, int nb, const float* __restrict__ W,
                                               const float* __restrict__ in, int nsplit, size_t split_stride,
                                               float* __restrict__ out, const int* __restrict__ xflag) {
    constexpr int T = NOUT / 16, NCP = T % 2 == 0 ? 2 : 1, CPW = T / NCP;   // column parts, tiles per wave
    static_assert(NIN % 32 == 0 && NOUT % 16 == 0, "tile");
    __builtin_amdgcn_s_setprio(2);   // issue ahead of the near-field waves sharing the SIMD
    const int item = blockIdx.x * 4 + int(threadIdx.x >> 6);
    const int g = item / NCP, cp = item % NCP;
    const int row0 = b0 + 16 * g, end = b0 + nb;
    if (row0 >= end) return;   // whole wave (no barrier in this kernel)
    const int lane = threadIdx.x & 63, i = lane & 15, kk = lane >> 4;
    const bool live = row0 + i < end;
    const float* arow = in + size_t(row0 + i) * NIN + 4 * kk;
    const float* wrow = W + size_t(16 * cp * CPW + i) * NIN + 4 * kk;
    v4f c[CPW];
#pragma unroll
    for (int t = 0; t < CPW; ++t) c[t] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < NIN; k0 += 32) {
        // two chunks per step: a box row's 128 contiguous bytes in one go
        float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0;
        if (live)
            for (int sp = 0; sp < nsplit; ++sp) {
                const float4 x0 = *reinterpret_cast<const float4*>(arow + sp * split_stride + k0);
                const float4 x1 = *reinterpret_cast<const float4*>(arow + sp * split_stride + k0 + 16);
                a0.x += x0.x; a0.y += x0.y; a0.z += x0.z; a0.w += x0.w;
                a1.x += x1.x; a1.y += x1.y; a1.z += x1.z; a1.w += x1.w;
            }
#pragma unroll
        for (int t = 0; t < CPW; ++t) {
            const float4 w0 = *reinterpret_cast<const float4*>(wrow + size_t(16 * t) * NIN + k0);
            const float4 w1 = *reinterpret_cast<const float4*>(wrow + size_t(16 * t) * NIN + k0 + 16);
            c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.x, w0.x, c[t], 0, 0, 0);
            c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.y, w0.y, c[t], 0, 0, 0);
            c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.z, w0.z, c[t], 0, 0, 0);
            c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.w, w0.w, c[t], 0, 0, 0);
            c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.x, w1.x, c[t], 0, 0, 0);
            c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.y, w1.y, c[t], 0, 0, 0);
            c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.z, w1.z, c[t], 0, 0, 0);
            c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.w, w1.w, c[t], 0, 0, 0);
        }
    }
    // D[4 kk + v][i] of tile t: box row0 + 4 kk + v, column 16 (cp CPW + t) + i
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int b = row0 + 4 * kk + v;
        if (b >= end) continue;
        float* o = out + size_t(b) * NOUT + 16 * cp * CPW + i;
        const bool add = ACCUM && xflag[b];
#pragma unroll
        for (int t = 0; t < CPW; ++t) o[16 * t] = add ? o[16 * t] + c[t][v] : c[t][v];
    }
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

constexpr int M2L_CB = 2;
constexpr int M2L_SPLIT = kM2LSplit;

const VOps* vops_device() {
    static DBuf* d = nullptr;
    if (!d) {
        d = new DBuf();
        d->ensure(sizeof(VOps));
        KIFMM_HIP(hipMemcpy(d->p, &vops_host(), sizeof(VOps), hipMemcpyHostToDevice));
    }
    return d->as<VOps>();
}

// Coarsest level with V lists: 2 in free space, 1 when periodic (the children
// of the root see the images of its neighbours); the root itself then
// receives the farther images through the lattice operator.
int first_v_level(const kifmm_plan* P) { return P->periodic ? 1 : 2; }
int first_down_level(const kifmm_plan* P) { return P->periodic ? 0 : 2; }

// M2L for all levels; nrhs = 2 treats densities rhs 0 and 1 together (the
// two columns share the target, the source and the operator), otherwise the
// densities of right-hand side `rhs`.
// M2L at tile size NP (the surface size, or the padded rank of the compressed
// basis): sources src [rhs][B][NP], optional start values init (the X-list
// check potentials; null for zero), partials out [split][rhs][B][NP].
template <int NP>
void launch_m2l_tile(kifmm_plan* P, int nrhs, int rhs, hipStream_t s, const float* src, const float* init,
                     float* out, const uint4* ops_f32, const uint4* ops_bf16, const float* const* stk3) {
    const int depth = P->depth;
    const int lv = first_v_level(P);
    if (depth < lv) return;
    const int b2 = int(P->bfar);
    const int TG = M2L_CB / nrhs;
    const int per_block = WAVES * TG * 16;
    TaskTable tt{};
    int blocks = 0;
    for (int l = lv; l <= depth; ++l) {
        const LevelInfo& pl = P->lev[l - 1];
        int groups = nblk(pl.nl_count, per_block);
        tt.first[tt.nlev] = blocks;
        tt.level[tt.nlev] = l;
        tt.nl_start[tt.nlev] = int(pl.nl_start);
        tt.nl_count[tt.nlev] = int(pl.nl_count);
        tt.groups[tt.nlev] = groups;
        tt.nlev++;
        blocks += groups;
    }
    blocks *= 8;
    if (blocks == 0) return;
    // A small tree has few tiles: split the V slots further so that the chip
    // fills and each block's chain of operator chunks is shorter.
    int nsplit = M2L_SPLIT;
    while (nsplit < P->m2l_split_cap && blocks * nsplit < kM2LFill) nsplit *= 2;
    P->m2l_split_used = nsplit;
    const size_t stride = size_t(P->B) * NP;
    const size_t sstride = 2 * stride;
    const float* phi_u = src + size_t(rhs) * stride;
    const float* psi_d = init ? init + size_t(rhs) * stride : nullptr;
    float* psi_m = out + size_t(rhs) * stride;
    const int total = blocks * nsplit;
    const BoxGeom geo{{P->lo[0], P->lo[1], P->lo[2]}, P->side};
    const float* const none[3] = {nullptr, nullptr, nullptr};
    const float* const* s3 = stk3 ? stk3 : none;
#define KIFMM_M2L_LAUNCH(SPL, CBV, OPS, STKV)                                                                    \
    hipLaunchKernelGGL((k_m2l<NP, SPL, CBV, STKV>), dim3(total), dim3(WAVES * 64), 0, s, tt, total, blocks,     \
                       nsplit, nrhs, P->nonleaf.as<int>(), P->bx_child.as<int2>(), P->vdense.as<int>(), b2,     \
                       vops_device(), phi_u, psi_d, P->xflag.as<int>(), psi_m, stride, sstride, OPS,            \
                       P->bx_anchor.as<int4>(), geo, s3[0], s3[1], s3[2])
    const bool split = P->opt.precision == KIFMM_SPLIT_BF16;
    if (stk3) {
        if (nrhs != 2) throw Error(KIFMM_ERR_STATE, "the framed Stokes M2L takes the sweep's two right-hand sides");
        if (split) KIFMM_M2L_LAUNCH(true, M2L_CB, ops_bf16, true);
        else KIFMM_M2L_LAUNCH(false, M2L_CB, ops_f32, true);
    } else {
        if (split) KIFMM_M2L_LAUNCH(true, M2L_CB, ops_bf16, false);
        else KIFMM_M2L_LAUNCH(false, M2L_CB, ops_f32, false);
    }
#undef KIFMM_M2L_LAUNCH
}

// sf: right-hand side `rhs` is the Stokeslet's fourth charge in per-box frames
template <int NP>
void launch_m2l(kifmm_plan* P, int nrhs, int rhs, hipStream_t s, const StokesFrames* sf = nullptr) {
    if (!P->cm) {
        const Operators& op = *P->ops;
        launch_m2l_tile<NP>(P, nrhs, rhs, s, P->phi_u.as<float>(), P->psi_d.as<float>(), P->psi_m.as<float>(),
                            op.m2l_f32.as<uint4>(), op.m2l_bf16.as<uint4>(), sf ? sf->up : nullptr);
        return;
    }
    const M2LBasis& cm = *P->cm;
#define KIFMM_M2L_TILE(KP)                                                                                     \
    launch_m2l_tile<KP>(P, nrhs, rhs, s, P->phi_k.as<float>(), nullptr, P->psi_m.as<float>(),               \
                        cm.core_f32.as<uint4>(), cm.core_bf16.as<uint4>(), sf ? sf->kp : nullptr)
    switch (cm.kp) {
        case 32: KIFMM_M2L_TILE(32); break;
        case 64: KIFMM_M2L_TILE(64); break;
        case 128: KIFMM_M2L_TILE(128); break;
        case 160: KIFMM_M2L_TILE(160); break;
        case 224: KIFMM_M2L_TILE(224); break;
        default: throw Error(KIFMM_ERR_STATE, "unsupported compressed M2L size");
    }
#undef KIFMM_M2L_TILE
}

// Compressed M2L: project (phi_k = Q^T phi_u) or expand (psi_d += Q psi_k)
// the boxes from the first V level on, for right-hand side r.
template <int NP, int KP>
void project_expand_kp(kifmm_plan* P, bool project, int r, hipStream_t s) {
    const int lv = first_v_level(P);
    if (P->depth < lv) return;
    const int b0 = int(P->lev[lv].start), nb = int(P->B) - b0;
    if (nb <= 0) return;
    const M2LBasis& cm = *P->cm;
    const size_t sn = size_t(P->B) * NP, sk = size_t(P->B) * KP;
    // work items: 16 boxes by one of the (one or two) column parts, four per block
    const auto blocks = [&](int nout) {
        const int parts = (nout / 16) % 2 == 0 ? 2 : 1;
        return dim3(unsigned(nblk(int64_t(nblk(nb, 16)) * parts, 4)));
    };
    if (project)
        hipLaunchKernelGGL((k_basis<NP, KP, false>), blocks(KP), dim3(256), 0, s, b0, nb, cm.qt.as<float>(),
                           P->phi_u.as<float>() + r * sn, 1, size_t(0), P->phi_k.as<float>() + r * sk, nullptr);
    else
        hipLaunchKernelGGL((k_basis<KP, NP, true>), blocks(NP), dim3(256), 0, s, b0, nb, cm.q.as<float>(),
                           P->psi_m.as<float>() + r * sk, P->m2l_split_used, 2 * sk, P->psi_d.as<float>() + r * sn,
                           P->xflag.as<int>());
}

template <int NP>
void project_expand(kifmm_plan* P, bool project, int r, hipStream_t s) {
    // the basis is only used when its tile is smaller than the surface's
    const int kp = P->cm->kp;
    if constexpr (NP > 32) if (kp == 32) return project_expand_kp<NP, 32>(P, project, r, s);
    if constexpr (NP > 64) if (kp == 64) return project_expand_kp<NP, 64>(P, project, r, s);
    if constexpr (NP > 128) if (kp == 128) return project_expand_kp<NP, 128>(P, project, r, s);
    if constexpr (NP > 160) if (kp == 160) return project_expand_kp<NP, 160>(P, project, r, s);
    if constexpr (NP > 224) if (kp == 224) return project_expand_kp<NP, 224>(P, project, r, s);
    throw Error(KIFMM_ERR_STATE, "unsupported compressed M2L size");
}

// One sweep over the tree for the right-hand sides r0 .. r1-1: 0 = the
// charges (monopoles), 1 = the adjoint sources (monopoles dL/du, dipoles
// dL/dE).  With both, M2L carries the two columns through each operator load.
// `between` runs after P2M (the caller forks the near field there).
template <int NP>
void sweep_impl(kifmm_plan* P, int r0, int r1, hipStream_t s, bool rec, const std::function<void()>& between,
                const StokesFrames* sf) {
    const Operators& op = *P->ops;
    // right-hand side 1 of a Stokes sweep carries the fourth charge in per-box frames
    auto stk = [&](int r) { return sf != nullptr && r == 1; };
    const int4* anc = P->bx_anchor.as<int4>();
    const int B = int(P->B);
    const size_t stride = size_t(B) * NP;
    BoxGeom geo{{P->lo[0], P->lo[1], P->lo[2]}, P->side};
    const float4* pts = P->pts.as<float4>();
    const float4* surf = op.surf.as<float4>();
    const int depth = P->depth;
    const int ld = first_down_level(P);
    if (P->periodic) {
        // moments of every right-hand side for the closed-form part of the kernel
        for (int r = r0; r < r1; ++r) {
            hipLaunchKernelGGL(k_moments, dim3(kMomentBlocks), dim3(256), 0, s, int64_t(P->N), pts,
                               r ? P->src2.as<float4>() : nullptr, P->lo[0] + 0.5 * P->side,
                               P->lo[1] + 0.5 * P->side, P->lo[2] + 0.5 * P->side, P->mom_part.as<double>());
            hipLaunchKernelGGL(k_moments_sum, dim3(1), dim3(64), 0, s, P->mom_part.as<double>(), kMomentBlocks,
                               P->mom.as<double>() + 16 * r);
        }
    }
    if (depth < ld) {
        if (rec) record_phase(P, 0, s);
        between();
        if (rec) for (int k = 1; k < 5; ++k) record_phase(P, k, s);
        return;
    }
    const int b2 = int(P->bfar);
    const int tpb = 2 * NP;   // P2M / P2L: two slices of NP threads
    // P2M
    for (int r = r0; r < r1; ++r)
        hipLaunchKernelGGL(k_p2m<NP>, dim3(unsigned(P->nleaves)), dim3(tpb), 0, s, P->leaves.as<int>(),
                           int(P->nleaves), b2, P->bx_anchor.as<int4>(), P->bx_range.as<int2>(), pts,
                           (r && !stk(r)) ? P->src2.as<float4>() : nullptr, stk(r) ? sf->frc : nullptr, surf, op.n,
                           geo, P->psi_u.as<float>() + r * stride);
    if (rec) record_phase(P, 0, s);
    between();
    // upward UC2E of the leaves (every level from ld in one launch), then
    // M2M + UC2E of the non-leaves, deepest level first; a column block holds
    // leaves only or non-leaves only, so no leaf waits on the M2M terms of
    // the children of others
    int64_t lf0 = 0;   // leaves above level ld, at the front of the leaf list
    for (int l = 0; l < ld; ++l) lf0 += P->lev[l].count - P->lev[l].nl_count;
    const int nlf = int(P->nleaves - lf0);
    for (int r = r0; r < r1; ++r) {
        auto up = [&](const int* list, int b0, int nb, bool shift) {
            const int blocks = nblk(nb, 16);
            if (blocks == 0) return;
#define KIFMM_UP(STKV, S0, S1, S2)                                                                                 \
    hipLaunchKernelGGL((k_updown<NP, true, STKV>), dim3(blocks), dim3(WAVES * 64), 0, s, blocks, b0, nb, list, 0, 0, \
                       0, P->nonleaf.as<int>(), P->bx_child.as<int2>(), P->bx_leaf.as<int>(),                       \
                       P->psi_u.as<float>() + r * stride, 1, size_t(0), P->phi_u.as<float>() + r * stride,         \
                       P->phi_u.as<float>() + r * stride, op.m2m.as<uint4>(), op.uc2e_w1.as<uint4>(),               \
                       op.uc2e_v.as<uint4>(), anc, geo, S0, S1, S2)
            if (shift) KIFMM_UP(true, sf->up[0], sf->up[1], sf->up[2]);
            else KIFMM_UP(false, (const float*)nullptr, (const float*)nullptr, (const float*)nullptr);
#undef KIFMM_UP
        };
        up(P->leaves.as<int>(), int(lf0), nlf, false);
        for (int l = depth; l >= ld; --l)
            up(P->nonleaf.as<int>(), int(P->lev[l].nl_start), int(P->lev[l].nl_count), stk(r));
    }
    // periodic root: every image beyond the root's neighbours
    if (P->periodic) {
        const DBuf& R = get_lattice_operator(P->p, P->opt.pinv_rtol);
        for (int r = r0; r < r1; ++r)
            hipLaunchKernelGGL(k_lattice, dim3(1), dim3(NP), 0, s, R.as<double>(), op.n, NP,
                               P->phi_u.as<float>() + r * stride, P->phi_d.as<float>() + r * stride);
    }
    // compressed M2L: its sources in the common basis
    if (P->cm)
        for (int r = r0; r < r1; ++r) project_expand<NP>(P, true, r, s);
    if (rec) record_phase(P, 1, s);
    // downward check potentials of the boxes the P2L kernel sums (flagged in
    // xflag; the M2L and the compressed expansion read no other box's value
    // before writing it)
    for (int r = r0; r < r1; ++r) {
        float* psi_d = P->psi_d.as<float>() + r * stride;
        if (P->n_xboxes > 0)
            hipLaunchKernelGGL(k_p2l<NP>, dim3(unsigned(P->n_xboxes)), dim3(tpb), 0, s, P->xboxes.as<int>(),
                               P->x_off.as<int>(), P->x_idx.as<int>(), P->bx_anchor.as<int4>(),
                               P->bx_range.as<int2>(), pts, (r && !stk(r)) ? P->src2.as<float4>() : nullptr,
                               stk(r) ? sf->frc : nullptr, surf, op.n, geo, psi_d);
    }
    if (rec) record_phase(P, 2, s);
    // V list (a Stokes sweep's second right-hand side in per-box frames)
    if (sf && (r0 != 0 || r1 != 2)) throw Error(KIFMM_ERR_STATE, "a Stokes sweep has right-hand sides 0 and 1");
    if (r1 - r0 == 2) {
        launch_m2l<NP>(P, 2, 0, s, sf);
    } else {
        for (int r = r0; r < r1; ++r) launch_m2l<NP>(P, 1, r, s);
    }
    if (rec) record_phase(P, 3, s);
    // compressed M2L: its results back on the check surfaces, added to the X
    // list (timed with the downward pass)
    if (P->cm)
        for (int r = r0; r < r1; ++r) project_expand<NP>(P, false, r, s);
    // L2L + DC2E, coarse to fine
    for (int r = r0; r < r1; ++r)
        for (int l = first_v_level(P); l <= depth; ++l) {
            const LevelInfo& pl = P->lev[l - 1];
            const int blocks = nblk(pl.nl_count, 16) * 8;
            if (blocks == 0) continue;
#define KIFMM_DOWN(STKV, S0, S1, S2)                                                                              \
    hipLaunchKernelGGL((k_updown<NP, false, STKV>), dim3(blocks), dim3(WAVES * 64), 0, s, blocks, 0, 0,           \
                       (const int*)nullptr, int(pl.nl_start), int(pl.nl_count), l > ld ? 1 : 0,                    \
                       P->nonleaf.as<int>(), P->bx_child.as<int2>(), P->bx_leaf.as<int>(),                         \
                       P->cm ? P->psi_d.as<float>() + r * stride : P->psi_m.as<float>() + r * stride,              \
                       P->cm ? 1 : P->m2l_split_used, 2 * stride, P->phi_d.as<float>() + r * stride,               \
                       P->phi_d.as<float>() + r * stride, op.l2l.as<uint4>(), op.dc2e_w1.as<uint4>(),              \
                       op.dc2e_v.as<uint4>(), anc, geo, S0, S1, S2)
            // the check potentials: M2L partials (with the X list in the first), or,
            // compressed, the expanded sum already in psi_d
            if (stk(r)) KIFMM_DOWN(true, sf->dn[0], sf->dn[1], sf->dn[2]);
            else KIFMM_DOWN(false, (const float*)nullptr, (const float*)nullptr, (const float*)nullptr);
#undef KIFMM_DOWN
        }
    if (rec) record_phase(P, 4, s);
}

template <int NP>
void far_impl(kifmm_plan* P, bool bwd, float* out_a, float* out_b, hipStream_t s, int rhs, bool acc, bool near,
              const StokesFrames* sf, bool sorted) {
    const Operators& op = *P->ops;
    BoxGeom geo{{P->lo[0], P->lo[1], P->lo[2]}, P->side};
    const int b2 = int(P->bfar);
    FarOut fo{near ? P->nearv.as<float4>() : nullptr, sorted ? nullptr : P->perm.as<int>(), out_a, out_b, nullptr,
              {0, 0, 0}, 0.0, acc ? 1 : 0, {nullptr, nullptr, nullptr}};
    if (sf)
        for (int d = 0; d < 3; ++d) fo.wsh[d] = sf->up[d];
    if (P->periodic) {
        fo.mom = P->mom.as<double>() + (bwd ? 0 : 16 * rhs);
        for (int d = 0; d < 3; ++d) fo.o[d] = P->lo[d] + 0.5 * P->side;
        fo.k1 = 2.0 * M_PI * P->c / (3.0 * P->side * P->side * P->side);
    }
    size_t stride = size_t(P->B) * NP;
    if (bwd)
        hipLaunchKernelGGL((k_far<NP, true>), dim3(unsigned(P->n_items)), dim3(256), 0, s, P->items_far.as<int2>(), b2,
                           P->bx_anchor.as<int4>(), P->bx_range.as<int2>(), P->wf_off.as<int>(), P->wf_idx.as<int>(),
                           P->pts.as<float4>(), P->src2.as<float4>(), P->phi_d.as<float>(), P->phi_u.as<float>(),
                           stride, op.surf.as<float4>(), op.n, geo, float(P->c), P->N, fo);
    else
        hipLaunchKernelGGL((k_far<NP, false>), dim3(unsigned(P->n_items)), dim3(256), 0, s, P->items_far.as<int2>(), b2,
                           P->bx_anchor.as<int4>(), P->bx_range.as<int2>(), P->wf_off.as<int>(), P->wf_idx.as<int>(),
                           P->pts.as<float4>(), (const float4*)nullptr, P->phi_d.as<float>() + rhs * stride,
                           P->phi_u.as<float>() + rhs * stride, stride, op.surf.as<float4>(), op.n, geo, float(P->c),
                           P->N, fo);
}

template <int NP>
void far_grad_impl(kifmm_plan* P, float* pot, float* field, float* grad, hipStream_t s, int rhs) {
    const Operators& op = *P->ops;
    BoxGeom geo{{P->lo[0], P->lo[1], P->lo[2]}, P->side};
    FarOut fo{P->nearv.as<float4>(), P->perm.as<int>(), pot, field, nullptr, {0, 0, 0}, 0.0, 0, {nullptr, nullptr, nullptr}};
    if (P->periodic) {
        fo.mom = P->mom.as<double>() + 16 * rhs;
        for (int d = 0; d < 3; ++d) fo.o[d] = P->lo[d] + 0.5 * P->side;
        fo.k1 = 2.0 * M_PI * P->c / (3.0 * P->side * P->side * P->side);
    }
    const size_t stride = size_t(P->B) * NP;
    hipLaunchKernelGGL((k_far_grad<NP>), dim3(unsigned(P->n_items)), dim3(256), 0, s, P->items_far.as<int2>(),
                       int(P->bfar), P->bx_anchor.as<int4>(), P->bx_range.as<int2>(), P->wf_off.as<int>(),
                       P->wf_idx.as<int>(), P->pts.as<float4>(), P->phi_d.as<float>() + rhs * stride,
                       P->phi_u.as<float>() + rhs * stride, op.surf.as<float4>(), op.n, geo, float(P->c), fo,
                       P->nearg.as<float>(), grad);
}

}  // namespace

namespace {
// Offset of every sorted point from the centre of its leaf (FP64, then FP32):
// the frame of the fourth harmonic charge at the targets.
__global__ __launch_bounds__(256) void k_stokes_frames(const int* __restrict__ leaves, const int4* __restrict__ anchor,
                                                       const int2* __restrict__ range, const int* __restrict__ perm,
                                                       const double* __restrict__ x64, BoxGeom geo,
                                                       float4* __restrict__ frame) {
    const int b = leaves[blockIdx.x];
    const int4 a = anchor[b];
    const int2 r = range[b];
    const double wd = ldexp(geo.side, -a.w);
    const double c0 = geo.lo[0] + (double(a.x) + 0.5) * wd, c1 = geo.lo[1] + (double(a.y) + 0.5) * wd,
                 c2 = geo.lo[2] + (double(a.z) + 0.5) * wd;
    for (int i = r.x + threadIdx.x; i < r.y; i += 256) {
        const size_t j = size_t(perm[i]);
        frame[i] = make_float4(float(x64[3 * j] - c0), float(x64[3 * j + 1] - c1), float(x64[3 * j + 2] - c2), 0.f);
    }
}

// Stokeslet velocity from the four harmonic charges' potentials psi_k and
// fields E(k) (the fourth about each target's leaf centre) and the near part,
// all in sorted order, written in caller order:
//   u_a = cf (psi_a + x'_k E(k)_a - E(4)_a) + near_a,  x' = x - (leaf centre),
// and, when p is set, the pressure p = cpf (E(1)_x + E(2)_y + E(3)_z) + cpn near_w.
__global__ void k_stokes_combine(int64_t N, const int* __restrict__ perm, const float4* __restrict__ frame,
                                 const float* __restrict__ pot, const float* __restrict__ fld,
                                 const float4* __restrict__ near, float cf, float cpf, float cpn,
                                 float* __restrict__ u, float* __restrict__ p) {
    int64_t i = blockIdx.x * int64_t(256) + threadIdx.x;
    if (i >= N) return;
    const size_t j = size_t(perm[i]);
    const float4 fr = frame[i];
    const float xp[3] = {fr.x, fr.y, fr.z};
    const float4 nr = near[i];
    const float na[3] = {nr.x, nr.y, nr.z};
    const size_t sN = size_t(N);
    for (int a = 0; a < 3; ++a) {
        float v = pot[a * sN + i] - fld[(3 * sN + i) * 3 + a];
        for (int k = 0; k < 3; ++k) v += xp[k] * fld[(k * sN + i) * 3 + a];
        u[3 * j + a] = cf * v + na[a];
    }
    if (p) p[j] = cpf * ((fld[3 * i] + fld[(sN + i) * 3 + 1]) + fld[(2 * sN + i) * 3 + 2]) + cpn * nr.w;
}
}  // namespace

void launch_stokes_frames(kifmm_plan* P, hipStream_t s) {
    P->stk_frame.ensure(size_t(P->N) * 16);
    const BoxGeom geo{{P->lo[0], P->lo[1], P->lo[2]}, P->side};
    if (P->nleaves > 0)
        hipLaunchKernelGGL(k_stokes_frames, dim3(unsigned(P->nleaves)), dim3(256), 0, s, P->leaves.as<int>(),
                           P->bx_anchor.as<int4>(), P->bx_range.as<int2>(), P->perm.as<int>(), P->x64.as<double>(),
                           geo, P->stk_frame.as<float4>());
}

void launch_stokes_combine(kifmm_plan* P, double viscosity, float* velocity, float* pressure, hipStream_t s) {
    const int64_t N = P->N;
    const float* pot = P->stk_far.as<float>();
    const float* fld = pot + 4 * size_t(N);
    hipLaunchKernelGGL(k_stokes_combine, dim3(unsigned((N + 255) / 256)), dim3(256), 0, s, N, P->perm.as<int>(),
                       P->stk_frame.as<float4>(), pot, fld, P->stk_near.as<float4>(),
                       float(1.0 / (8.0 * M_PI * viscosity * P->c)), float(1.0 / (4.0 * M_PI * P->c)),
                       float(1.0 / (4.0 * M_PI)), velocity, pressure);
}

void run_far_grad(kifmm_plan* P, float* pot, float* field, float* grad, hipStream_t s, int rhs) {
    switch (P->npad) {
        case 32: far_grad_impl<32>(P, pot, field, grad, s, rhs); break;
        case 64: far_grad_impl<64>(P, pot, field, grad, s, rhs); break;
        case 128: far_grad_impl<128>(P, pot, field, grad, s, rhs); break;
        case 160: far_grad_impl<160>(P, pot, field, grad, s, rhs); break;
        case 224: far_grad_impl<224>(P, pot, field, grad, s, rhs); break;
        case 320: far_grad_impl<320>(P, pot, field, grad, s, rhs); break;
        default: throw Error(KIFMM_ERR_ARG, "unsupported surface size");
    }
}

void run_sweep(kifmm_plan* P, int r0, int r1, hipStream_t s, bool record, const std::function<void()>& between,
               const StokesFrames* sf) {
    switch (P->npad) {
        case 32: sweep_impl<32>(P, r0, r1, s, record, between, sf); break;
        case 64: sweep_impl<64>(P, r0, r1, s, record, between, sf); break;
        case 128: sweep_impl<128>(P, r0, r1, s, record, between, sf); break;
        case 160: sweep_impl<160>(P, r0, r1, s, record, between, sf); break;
        case 224: sweep_impl<224>(P, r0, r1, s, record, between, sf); break;
        case 320: sweep_impl<320>(P, r0, r1, s, record, between, sf); break;
        default: throw Error(KIFMM_ERR_ARG, "unsupported surface size");
    }
}

void run_far_eval(kifmm_plan* P, bool backward, float* out_a, float* out_b, hipStream_t s, int rhs, bool acc,
                  bool near, const StokesFrames* sf, bool sorted) {
    switch (P->npad) {
        case 32: far_impl<32>(P, backward, out_a, out_b, s, rhs, acc, near, sf, sorted); break;
        case 64: far_impl<64>(P, backward, out_a, out_b, s, rhs, acc, near, sf, sorted); break;
        case 128: far_impl<128>(P, backward, out_a, out_b, s, rhs, acc, near, sf, sorted); break;
        case 160: far_impl<160>(P, backward, out_a, out_b, s, rhs, acc, near, sf, sorted); break;
        case 224: far_impl<224>(P, backward, out_a, out_b, s, rhs, acc, near, sf, sorted); break;
        case 320: far_impl<320>(P, backward, out_a, out_b, s, rhs, acc, near, sf, sorted); break;
        default: throw Error(KIFMM_ERR_ARG, "unsupported surface size");
    }
}

}  // namespace kifmm
