// Near field (Section 2.2, last step: the contributions of points in the near
// zone) and the final combination with the far field.
//
// One block per target leaf, one target per lane.  The U-list source leaves
// are staged through LDS as float4 (x, y, z, q) in global FP32 coordinates, so
// every pair difference is a correctly rounded FP32 subtraction of the input
// coordinates; pairs at distance exactly zero (the self pair, coincident
// points) are skipped.  The forward kernel counts 20 FLOP per pair (3 sub,
// 5 for r^2, rsqrt, 4 for 1/r and 1/r^3 with q, 7 for the four sums).
#include "common.h"

namespace kifmm {

namespace {

constexpr int P2P_THREADS = 128;
constexpr int P2P_STAGE = 256;

__global__ void k_gather(int64_t N, const float4* __restrict__ xs, const int* __restrict__ perm,
                         const float* __restrict__ q, float4* __restrict__ pts) {
    int64_t i = blockIdx.x * int64_t(256) + threadIdx.x;
    if (i >= N) return;
    float4 x = xs[i];
    x.w = q[perm[i]];
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

__global__ __launch_bounds__(P2P_THREADS) void k_p2p(const int* __restrict__ leaves, const int2* __restrict__ range,
                                                     const int* __restrict__ uoff, const int* __restrict__ uidx,
                                                     const float4* __restrict__ pts, const float4* __restrict__ far,
                                                     const int* __restrict__ perm, float cst,
                                                     float* __restrict__ pot, float* __restrict__ field) {
    __shared__ float4 sh[P2P_STAGE];
    const int b = leaves[blockIdx.x];
    const int2 r = range[b];
    for (int t0 = r.x; t0 < r.y; t0 += P2P_THREADS) {
        const int i = t0 + threadIdx.x;
        const bool act = i < r.y;
        const float4 x = act ? pts[i] : make_float4(0, 0, 0, 0);
        float u = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
        for (int k = uoff[b]; k < uoff[b + 1]; ++k) {
            const int2 ra = range[uidx[k]];
            for (int s0 = ra.x; s0 < ra.y; s0 += P2P_STAGE) {
                const int m = min(P2P_STAGE, ra.y - s0);
                __syncthreads();
                for (int j = threadIdx.x; j < m; j += P2P_THREADS) sh[j] = pts[s0 + j];
                __syncthreads();
#pragma unroll 4
                for (int j = 0; j < m; ++j) {
                    const float4 y = sh[j];
                    const float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z;
                    const float ri = rsq(dx * dx + dy * dy + dz * dz);
                    const float qr = y.w * ri;
                    const float qr3 = qr * ri * ri;
                    u += qr;
                    ex += qr3 * dx;
                    ey += qr3 * dy;
                    ez += qr3 * dz;
                }
            }
        }
        if (act) {
            const float4 f = far[i];
            const int j = perm[i];
            if (pot) pot[j] = f.x + cst * u;
            if (field) {
                field[3 * size_t(j)] = f.y + cst * ex;
                field[3 * size_t(j) + 1] = f.z + cst * ey;
                field[3 * size_t(j) + 2] = f.w + cst * ez;
            }
        }
    }
}

// Backward near field and the combination
//   qbar_k = psi_k,  xbar_k = -ubar_k E_k - H_k Ebar_k - q_k E_psi,k
// where E, H come from the charges q and psi, E_psi from monopoles ubar and
// dipoles Ebar (psi = sum ubar K - Ebar . G).
__global__ __launch_bounds__(P2P_THREADS) void k_p2p_bwd(const int* __restrict__ leaves, const int2* __restrict__ range,
                                                         const int* __restrict__ uoff, const int* __restrict__ uidx,
                                                         const float4* __restrict__ pts, const float4* __restrict__ src2,
                                                         const float* __restrict__ far, int64_t N,
                                                         const int* __restrict__ perm, float cst,
                                                         float* __restrict__ gq, float* __restrict__ gx) {
    __shared__ float4 sh[P2P_STAGE];
    __shared__ float4 sh2[P2P_STAGE];
    const int b = leaves[blockIdx.x];
    const int2 r = range[b];
    for (int t0 = r.x; t0 < r.y; t0 += P2P_THREADS) {
        const int i = t0 + threadIdx.x;
        const bool act = i < r.y;
        const float4 x = act ? pts[i] : make_float4(0, 0, 0, 0);
        const float4 a = act ? src2[i] : make_float4(0, 0, 0, 0);
        float e1x = 0, e1y = 0, e1z = 0, hx = 0, hy = 0, hz = 0, ps = 0, px = 0, py = 0, pz = 0;
        for (int k = uoff[b]; k < uoff[b + 1]; ++k) {
            const int2 ra = range[uidx[k]];
            for (int s0 = ra.x; s0 < ra.y; s0 += P2P_STAGE) {
                const int m = min(P2P_STAGE, ra.y - s0);
                __syncthreads();
                for (int j = threadIdx.x; j < m; j += P2P_THREADS) {
                    sh[j] = pts[s0 + j];
                    sh2[j] = src2[s0 + j];
                }
                __syncthreads();
                for (int j = 0; j < m; ++j) {
                    const float4 y = sh[j];
                    const float4 bj = sh2[j];
                    const float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z;
                    const float ri = rsq(dx * dx + dy * dy + dz * dz);
                    const float ri3 = ri * ri * ri;
                    const float ri5 = ri3 * ri * ri;
                    // field of q_j and H(r) Ebar_k
                    const float g = y.w * ri3;
                    e1x += g * dx;
                    e1y += g * dy;
                    e1z += g * dz;
                    const float rk = dx * a.y + dy * a.z + dz * a.w;
                    const float h3 = 3.f * y.w * rk * ri5;
                    hx += h3 * dx - g * a.y;
                    hy += h3 * dy - g * a.z;
                    hz += h3 * dz - g * a.w;
                    // psi and E_psi of (ubar_j, Ebar_j):  psi = ubar K - Ebar.G,
                    // E_psi = ubar G - H Ebar
                    const float rj = dx * bj.y + dy * bj.z + dz * bj.w;
                    ps += bj.x * ri - rj * ri3;
                    const float g2 = bj.x * ri3;
                    const float h2 = 3.f * rj * ri5;
                    px += g2 * dx - (h2 * dx - bj.y * ri3);
                    py += g2 * dy - (h2 * dy - bj.z * ri3);
                    pz += g2 * dz - (h2 * dz - bj.w * ri3);
                }
            }
        }
        if (act) {
            const float E1x = far[0 * N + i] + cst * e1x, E1y = far[1 * N + i] + cst * e1y,
                        E1z = far[2 * N + i] + cst * e1z;
            const float Hx = far[3 * N + i] + cst * hx, Hy = far[4 * N + i] + cst * hy, Hz = far[5 * N + i] + cst * hz;
            const float Ps = far[6 * N + i] + cst * ps;
            const float Px = far[7 * N + i] + cst * px, Py = far[8 * N + i] + cst * py, Pz = far[9 * N + i] + cst * pz;
            const int j = perm[i];
            if (gq) gq[j] = Ps;
            if (gx) {
                gx[3 * size_t(j)] = -a.x * E1x - Hx - x.w * Px;
                gx[3 * size_t(j) + 1] = -a.x * E1y - Hy - x.w * Py;
                gx[3 * size_t(j) + 2] = -a.x * E1z - Hz - x.w * Pz;
            }
        }
    }
}

}  // namespace

void launch_gather(kifmm_plan* P, const float* charges, const float* gpot, const float* gfield, bool adjoint,
                   hipStream_t s) {
    const int64_t N = P->N;
    P->pts.ensure(size_t(N) * 16);
    hipLaunchKernelGGL(k_gather, dim3(unsigned((N + 255) / 256)), dim3(256), 0, s, N, P->xs.as<float4>(),
                       P->perm.as<int>(), charges, P->pts.as<float4>());
    if (adjoint) {
        P->src2.ensure(size_t(N) * 16);
        hipLaunchKernelGGL(k_gather_adj, dim3(unsigned((N + 255) / 256)), dim3(256), 0, s, N, P->perm.as<int>(), gpot,
                           gfield, P->src2.as<float4>());
    }
}

void launch_p2p_forward(kifmm_plan* P, float* potential, float* field, hipStream_t s) {
    hipLaunchKernelGGL(k_p2p, dim3(unsigned(P->nleaves)), dim3(P2P_THREADS), 0, s, P->leaves.as<int>(),
                       P->bx_range.as<int2>(), P->u_off.as<int>(), P->u_idx.as<int>(), P->pts.as<float4>(),
                       P->far.as<float4>(), P->perm.as<int>(), float(P->c), potential, field);
}

void launch_p2p_backward(kifmm_plan* P, float* gq, float* gx, hipStream_t s) {
    hipLaunchKernelGGL(k_p2p_bwd, dim3(unsigned(P->nleaves)), dim3(P2P_THREADS), 0, s, P->leaves.as<int>(),
                       P->bx_range.as<int2>(), P->u_off.as<int>(), P->u_idx.as<int>(), P->pts.as<float4>(),
                       P->src2.as<float4>(), P->far.as<float>(), P->N, P->perm.as<int>(), float(P->c), gq, gx);
}

}  // namespace kifmm
