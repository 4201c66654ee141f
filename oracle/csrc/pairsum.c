/*
 * Oracle helper: plain FP64 pair sums for the 1/r kernel.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is part of the CPU oracle that checks
 * the GPU library; it is never linked into the library.
 *
 * Kernel (the paper's eq. (1) specialised to the Laplace potential of eq. (3)
 * and the gravitational potential of eq. (4)):
 *     K(r) = c / |r|,           r = x_target - y_source
 *     G(r) = -grad K = c r / |r|^3
 *     H(r) = grad grad K = c (3 r r^T / |r|^5 - I / |r|^3)
 * A source j carries a monopole s_j and optionally a dipole m_j; the field it
 * makes is  psi(x) = s_j K(r) - m_j . G(r).  Outputs at a target are
 *     u = psi,   E = -grad psi = s_j G(r) - H(r) m_j,   Hess = grad grad psi,
 * the dipole part of the Hessian being the derivative of -m . G:
 *     c [3 (m_a r_b + m_b r_a + (m.r) delta_ab) / |r|^5 - 15 (m.r) r_a r_b / |r|^7].
 * Pairs at distance exactly zero (the self pair and coincident points) are
 * skipped.
 *
 * Everything is a straight double loop; OpenMP only splits the targets.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

static void one_pair(const double* xt, const double* ys, double s, const double* m, double c,
                     double* u, double* e, double* h)
{
    double r0 = xt[0] - ys[0], r1 = xt[1] - ys[1], r2 = xt[2] - ys[2];
    double rr = r0 * r0 + r1 * r1 + r2 * r2;
    if (rr == 0.0) return;
    double ri = 1.0 / sqrt(rr);
    double ri3 = ri * ri * ri;
    double ri5 = ri3 * ri * ri;
    /* monopole */
    *u += c * s * ri;
    e[0] += c * s * r0 * ri3;
    e[1] += c * s * r1 * ri3;
    e[2] += c * s * r2 * ri3;
    if (h) {
        h[0] += c * s * (3.0 * r0 * r0 * ri5 - ri3);
        h[1] += c * s * (3.0 * r1 * r1 * ri5 - ri3);
        h[2] += c * s * (3.0 * r2 * r2 * ri5 - ri3);
        h[3] += c * s * (3.0 * r0 * r1 * ri5);
        h[4] += c * s * (3.0 * r0 * r2 * ri5);
        h[5] += c * s * (3.0 * r1 * r2 * ri5);
    }
    /* dipole: psi = -m.G(r);  E = -grad psi = -H(r) m */
    if (m) {
        double mr = m[0] * r0 + m[1] * r1 + m[2] * r2;
        *u -= c * mr * ri3;
        e[0] -= c * (3.0 * r0 * mr * ri5 - m[0] * ri3);
        e[1] -= c * (3.0 * r1 * mr * ri5 - m[1] * ri3);
        e[2] -= c * (3.0 * r2 * mr * ri5 - m[2] * ri3);
        if (h) {
            double ri7 = ri5 * ri * ri;
            double r[3] = {r0, r1, r2};
            static const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
            for (int k = 0; k < 6; ++k) {
                int a = A[k], b = B[k];
                double t = 3.0 * (m[a] * r[b] + m[b] * r[a] + (a == b ? mr : 0.0)) * ri5
                           - 15.0 * mr * r[a] * r[b] * ri7;
                h[k] += c * t;
            }
        }
    }
}

/* Direct sum: every target against every source. */
void oracle_direct(int64_t nt, const double* xt, int64_t ns, const double* ys,
                   const double* s, const double* m, double c,
                   double* u, double* e, double* h)
{
    #pragma omp parallel for schedule(dynamic, 16) if (nt * ns > 200000)
    for (int64_t i = 0; i < nt; ++i) {
        double ui = 0.0, ei[3] = {0.0, 0.0, 0.0}, hi[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t j = 0; j < ns; ++j)
            one_pair(xt + 3 * i, ys + 3 * j, s[j], m ? m + 3 * j : NULL, c, &ui, ei, h ? hi : NULL);
        if (u) u[i] = ui;
        if (e) { e[3 * i] = ei[0]; e[3 * i + 1] = ei[1]; e[3 * i + 2] = ei[2]; }
        if (h) for (int k = 0; k < 6; ++k) h[6 * i + k] = hi[k];
    }
}

/* Near field over U lists.  Target t is point tidx[t] of the sorted arrays and
 * lies in leaf tleaf[t]; its sources are the points of every leaf A in
 * U(tleaf[t]) = uidx[uoff[tleaf[t]] .. uoff[tleaf[t]+1]), each leaf A holding
 * sorted points begin[A] .. end[A].  With periodic images, entry k of the
 * lists moves its leaf's points by ushift[3k .. 3k+2] (NULL: no shifts). */
void oracle_p2p(int64_t nt, const int64_t* tidx, const int64_t* tleaf,
                const int64_t* begin, const int64_t* end,
                const int64_t* uoff, const int64_t* uidx, const double* ushift,
                const double* x, const double* s, const double* m, double c,
                double* u, double* e, double* h)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nt; ++t) {
        const double* xt = x + 3 * tidx[t];
        int64_t L = tleaf[t];
        double ut = 0.0, et[3] = {0.0, 0.0, 0.0}, ht[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t k = uoff[L]; k < uoff[L + 1]; ++k) {
            int64_t A = uidx[k];
            for (int64_t j = begin[A]; j < end[A]; ++j) {
                double y[3] = {x[3 * j], x[3 * j + 1], x[3 * j + 2]};
                if (ushift) {
                    y[0] += ushift[3 * k];
                    y[1] += ushift[3 * k + 1];
                    y[2] += ushift[3 * k + 2];
                }
                one_pair(xt, y, s[j], m ? m + 3 * j : NULL, c, &ut, et, h ? ht : NULL);
            }
        }
        if (u) u[t] = ut;
        if (e) { e[3 * t] = et[0]; e[3 * t + 1] = et[1]; e[3 * t + 2] = et[2]; }
        if (h) for (int k = 0; k < 6; ++k) h[6 * t + k] = ht[k];
    }
}
