// Clump aggregation (Section 2.4): the long-range forces act on the pebbles
// and are summed, with their moments, into the force and torque of each clump.
// One thread per clump walks its pebbles in caller order and accumulates in
// FP64, so the result is deterministic.
#include "common.h"

namespace kifmm {

namespace {

__global__ void k_clump(int64_t C, const int64_t* __restrict__ off, const double* __restrict__ x,
                        const float* __restrict__ q, const float* __restrict__ E, const double* __restrict__ cen,
                        double* __restrict__ F, double* __restrict__ T) {
    int64_t c = blockIdx.x * int64_t(256) + threadIdx.x;
    if (c >= C) return;
    double fx = 0, fy = 0, fz = 0, tx = 0, ty = 0, tz = 0;
    const double X0 = cen[3 * c], X1 = cen[3 * c + 1], X2 = cen[3 * c + 2];
    for (int64_t k = off[c]; k < off[c + 1]; ++k) {
        const double qk = q[k];
        const double gx = qk * double(E[3 * k]), gy = qk * double(E[3 * k + 1]), gz = qk * double(E[3 * k + 2]);
        const double rx = x[3 * k] - X0, ry = x[3 * k + 1] - X1, rz = x[3 * k + 2] - X2;
        fx += gx;
        fy += gy;
        fz += gz;
        tx += ry * gz - rz * gy;
        ty += rz * gx - rx * gz;
        tz += rx * gy - ry * gx;
    }
    F[3 * c] = fx;
    F[3 * c + 1] = fy;
    F[3 * c + 2] = fz;
    T[3 * c] = tx;
    T[3 * c + 1] = ty;
    T[3 * c + 2] = tz;
}

// Backward of the clump aggregation for dL/dF_c = Fb, dL/dT_c = Tb (either may
// be null = 0), with r_k = x_k - X_c:
//   dL/dq_k = Fb.E_k + Tb.(r_k x E_k),  dL/dE_k = q_k (Fb + Tb x r_k),
//   dL/dx_k = q_k (E_k x Tb),           dL/dX_c = -sum_k dL/dx_k.
// One thread per clump, FP64 arithmetic, caller order (deterministic).
__global__ void k_clump_bwd(int64_t C, const int64_t* __restrict__ off, const double* __restrict__ x,
                            const float* __restrict__ q, const float* __restrict__ E,
                            const double* __restrict__ cen, const double* __restrict__ Fb,
                            const double* __restrict__ Tb, float* __restrict__ qb, float* __restrict__ Eb,
                            float* __restrict__ xb, double* __restrict__ Xb) {
    int64_t c = blockIdx.x * int64_t(256) + threadIdx.x;
    if (c >= C) return;
    const double f0 = Fb ? Fb[3 * c] : 0.0, f1 = Fb ? Fb[3 * c + 1] : 0.0, f2 = Fb ? Fb[3 * c + 2] : 0.0;
    const double t0 = Tb ? Tb[3 * c] : 0.0, t1 = Tb ? Tb[3 * c + 1] : 0.0, t2 = Tb ? Tb[3 * c + 2] : 0.0;
    const double X0 = cen[3 * c], X1 = cen[3 * c + 1], X2 = cen[3 * c + 2];
    double s0 = 0, s1 = 0, s2 = 0;
    for (int64_t k = off[c]; k < off[c + 1]; ++k) {
        const double qk = q[k];
        const double e0 = E[3 * k], e1 = E[3 * k + 1], e2 = E[3 * k + 2];
        const double r0 = x[3 * k] - X0, r1 = x[3 * k + 1] - X1, r2 = x[3 * k + 2] - X2;
        // r x E, Tb x r, E x Tb
        const double c0 = r1 * e2 - r2 * e1, c1 = r2 * e0 - r0 * e2, c2 = r0 * e1 - r1 * e0;
        const double d0 = t1 * r2 - t2 * r1, d1 = t2 * r0 - t0 * r2, d2 = t0 * r1 - t1 * r0;
        const double g0 = qk * (e1 * t2 - e2 * t1), g1 = qk * (e2 * t0 - e0 * t2), g2 = qk * (e0 * t1 - e1 * t0);
        if (qb) qb[k] = float((f0 * e0 + f1 * e1 + f2 * e2) + (t0 * c0 + t1 * c1 + t2 * c2));
        if (Eb) {
            Eb[3 * k] = float(qk * (f0 + d0));
            Eb[3 * k + 1] = float(qk * (f1 + d1));
            Eb[3 * k + 2] = float(qk * (f2 + d2));
        }
        if (xb) {
            xb[3 * k] = float(g0);
            xb[3 * k + 1] = float(g1);
            xb[3 * k + 2] = float(g2);
        }
        s0 += g0;
        s1 += g1;
        s2 += g2;
    }
    if (Xb) {
        Xb[3 * c] = -s0;
        Xb[3 * c + 1] = -s1;
        Xb[3 * c + 2] = -s2;
    }
}

// zero the per-pebble outputs of pebbles after the last clump
__global__ void k_zero_tail(int64_t from, int64_t N, float* __restrict__ qb, float* __restrict__ Eb,
                            float* __restrict__ xb) {
    int64_t k = from + blockIdx.x * int64_t(256) + threadIdx.x;
    if (k >= N) return;
    if (qb) qb[k] = 0.f;
    for (int d = 0; d < 3; ++d) {
        if (Eb) Eb[3 * k + d] = 0.f;
        if (xb) xb[3 * k + d] = 0.f;
    }
}

}  // namespace

void launch_clump_backward(kifmm_plan* P, const float* q, const float* E, const int64_t* off, int64_t C,
                           int64_t covered, const double* centers, const double* Fb, const double* Tb, float* qb,
                           float* Eb, float* xb, double* Xb, hipStream_t s) {
    if (C > 0)
        hipLaunchKernelGGL(k_clump_bwd, dim3(unsigned((C + 255) / 256)), dim3(256), 0, s, C, off,
                           P->x64.as<double>(), q, E, centers, Fb, Tb, qb, Eb, xb, Xb);
    if (covered < P->N)
        hipLaunchKernelGGL(k_zero_tail, dim3(unsigned((P->N - covered + 255) / 256)), dim3(256), 0, s, covered,
                           P->N, qb, Eb, xb);
}

void launch_clump_reduce(kifmm_plan* P, const float* q, const float* E, const int64_t* off, int64_t C,
                         const double* centers, double* F, double* T, hipStream_t s) {
    if (C <= 0) return;
    hipLaunchKernelGGL(k_clump, dim3(unsigned((C + 255) / 256)), dim3(256), 0, s, C, off, P->x64.as<double>(), q, E,
                       centers, F, T);
}

}  // namespace kifmm
