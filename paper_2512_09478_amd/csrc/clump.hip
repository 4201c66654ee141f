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

}  // namespace

void launch_clump_reduce(kifmm_plan* P, const float* q, const float* E, const int64_t* off, int64_t C,
                         const double* centers, double* F, double* T, hipStream_t s) {
    if (C <= 0) return;
    hipLaunchKernelGGL(k_clump, dim3(unsigned((C + 255) / 256)), dim3(256), 0, s, C, off, P->x64.as<double>(), q, E,
                       centers, F, T);
}

}  // namespace kifmm
