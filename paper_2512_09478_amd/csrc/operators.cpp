// FP64 operator precompute (host) and its upload to the device.
//
// Section 2.2 describes the far field of a box by a density on samples of an
// equivalent surface and the M2M, L2L and M2L operators as matrices computed
// automatically from the kernel.  Everything here is built once per (p, tau)
// in unit-box coordinates for the kernel 1/r; the homogeneity of 1/r makes
// the operators level independent (a box of side w scales K by 1/w, which the
// sweep folds into its normalised check potentials), and the kernel constant
// c cancels between a check potential and its pseudoinverse, so it is applied
// only to the final outputs.
//
// Surfaces: boundary points of the p^3 grid, rho = 1.05 (upward equivalent =
// downward check) and rho = 2.95 (upward check = downward equivalent).  With
// these the downward check-to-equivalent map is the transpose of the upward
// one, L2L is the transpose of M2M, and M2L(-d) = M2L(d)^T, which is what
// makes the transposed (adjoint) sweep reuse the forward operators.
//
// Check-to-equivalent: truncated SVD of K(uc, ue) (one-sided Jacobi, FP64),
// singular values below tau * sigma_1 dropped, applied in factored form
// V (Sigma^-1 U^T psi) so that FP32 rounding stays inside the kept subspace.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <tuple>

#include "common.h"

namespace kifmm {

std::vector<double> unit_surface(int p, double rho) {
    std::vector<double> out;
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
            for (int k = 0; k < p; ++k) {
                bool bnd = std::min(i, std::min(j, k)) == 0 || std::max(i, std::max(j, k)) == p - 1;
                if (!bnd) continue;
                out.push_back(rho * (double(i) / (p - 1) - 0.5));
                out.push_back(rho * (double(j) / (p - 1) - 0.5));
                out.push_back(rho * (double(k) / (p - 1) - 0.5));
            }
    return out;
}

void jacobi_svd(int n, const double* A, double* U, double* S, double* V) {
    // Columns of G = A V are rotated pairwise until mutually orthogonal; then
    // sigma_j = |g_j| and u_j = g_j / sigma_j.  Column-major working copies.
    std::vector<double> G(size_t(n) * n), W(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) G[size_t(j) * n + i] = A[size_t(i) * n + j];
    for (int j = 0; j < n; ++j) W[size_t(j) * n + j] = 1.0;
    for (int sweep = 0; sweep < 80; ++sweep) {
        int rotations = 0;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double* gp = &G[size_t(p) * n];
                double* gq = &G[size_t(q) * n];
                double a = 0, b = 0, g = 0;
                for (int i = 0; i < n; ++i) {
                    a += gp[i] * gp[i];
                    b += gq[i] * gq[i];
                    g += gp[i] * gq[i];
                }
                if (g == 0.0 || fabs(g) <= 1e-15 * sqrt(a * b)) continue;
                ++rotations;
                double zeta = (b - a) / (2.0 * g);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t);
                double sn = cs * t;
                for (int i = 0; i < n; ++i) {
                    double x = gp[i], y = gq[i];
                    gp[i] = cs * x - sn * y;
                    gq[i] = sn * x + cs * y;
                }
                double* wp = &W[size_t(p) * n];
                double* wq = &W[size_t(q) * n];
                for (int i = 0; i < n; ++i) {
                    double x = wp[i], y = wq[i];
                    wp[i] = cs * x - sn * y;
                    wq[i] = sn * x + cs * y;
                }
            }
        }
        if (rotations == 0) break;
    }
    std::vector<double> sig(n);
    for (int j = 0; j < n; ++j) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += G[size_t(j) * n + i] * G[size_t(j) * n + i];
        sig[j] = sqrt(s);
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return sig[a] > sig[b]; });
    for (int r = 0; r < n; ++r) {
        int j = ord[r];
        S[r] = sig[j];
        for (int i = 0; i < n; ++i) {
            U[size_t(i) * n + r] = sig[j] > 0 ? G[size_t(j) * n + i] / sig[j] : 0.0;
            V[size_t(i) * n + r] = W[size_t(j) * n + i];
        }
    }
}

namespace {

uint16_t bf16_rne(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return uint16_t(u >> 16);
}

float bf16_to_float(uint16_t h) {
    uint32_t u = uint32_t(h) << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

double inv_dist(const double* a, const double* b) {
    double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    return 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

void upload(DBuf& buf, const void* host, size_t bytes) {
    buf.ensure(bytes);
    KIFMM_HIP(hipMemcpy(buf.p, host, bytes, hipMemcpyHostToDevice));
}

// MFMA fragment order of an np x np row-major operator for the gathered
// products: chunk kc (32 columns), row block rb (16 rows), half h, lane l
// (row 16 rb + l%16, columns 32 kc + 8 (l/16) + ...).  FP32: half h holds
// columns +4h..+4h+3.  bf16: half 0 holds the 8 hi parts, half 1 the lo parts.
// Each (operator, chunk) is a contiguous block of np/16 * 128 16-byte words.
void frag_f32(const float* A, int np, uint32_t* out) {
    const int RB = np / 16, KC = np / 32;
    for (int kc = 0; kc < KC; ++kc)
        for (int rb = 0; rb < RB; ++rb)
            for (int h = 0; h < 2; ++h)
                for (int l = 0; l < 64; ++l) {
                    size_t w = ((size_t(kc) * RB + rb) * 2 + h) * 64 + l;
                    const float* src = A + size_t(rb * 16 + (l & 15)) * np + kc * 32 + 8 * (l >> 4) + 4 * h;
                    memcpy(out + 4 * w, src, 16);
                }
}

void frag_bf16(const uint16_t* hi, const uint16_t* lo, int np, uint16_t* out) {
    const int RB = np / 16, KC = np / 32;
    for (int kc = 0; kc < KC; ++kc)
        for (int rb = 0; rb < RB; ++rb)
            for (int h = 0; h < 2; ++h)
                for (int l = 0; l < 64; ++l) {
                    size_t w = ((size_t(kc) * RB + rb) * 2 + h) * 64 + l;
                    const uint16_t* src = (h ? lo : hi) + size_t(rb * 16 + (l & 15)) * np + kc * 32 + 8 * (l >> 4);
                    memcpy(out + 8 * w, src, 16);
                }
}

// Chain order of an np x np operator whose right factor is a result still in
// MFMA accumulator layout: output block ob, k block rb, lane l holds
// A[16 ob + l%16][16 rb + 4 (l/16) .. +3].  One output block is a contiguous
// chunk of np/16 * 64 16-byte words.
void frag_chain(const float* A, int np, uint32_t* out) {
    const int RB = np / 16;
    for (int ob = 0; ob < RB; ++ob)
        for (int rb = 0; rb < RB; ++rb)
            for (int l = 0; l < 64; ++l) {
                size_t w = (size_t(ob) * RB + rb) * 64 + l;
                memcpy(out + 4 * w, A + size_t(ob * 16 + (l & 15)) * np + rb * 16 + 4 * (l >> 4), 16);
            }
}

std::unique_ptr<Operators> build_operators(int p, double tau) {
    auto op = std::make_unique<Operators>();
    const int n = 6 * (p - 1) * (p - 1) + 2;
    const int np = (n + 31) / 32 * 32;
    op->p = p;
    op->n = n;
    op->npad = np;
    op->tau = tau;
    std::vector<double> sin = unit_surface(p, 1.05);   // ue = dc
    std::vector<double> sout = unit_surface(p, 2.95);  // uc = de

    // surfaces for the kernels
    std::vector<float> surf(size_t(2) * np * 4, 0.0f);
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            surf[size_t(i) * 4 + d] = float(sin[3 * i + d]);
            surf[size_t(np + i) * 4 + d] = float(sout[3 * i + d]);
        }
    upload(op->surf, surf.data(), surf.size() * 4);

    // K(uc, ue) and its truncated pseudoinverse, factored
    std::vector<double> K(size_t(n) * n), U(size_t(n) * n), V(size_t(n) * n), S(n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) K[size_t(i) * n + j] = inv_dist(&sout[3 * i], &sin[3 * j]);
    jacobi_svd(n, K.data(), U.data(), S.data(), V.data());
    int k = 0;
    while (k < n && S[k] >= tau * S[0]) ++k;
    op->rank = k;
    op->sigma.assign(S.begin(), S.end());
    op->svd_u = U;
    op->svd_v = V;
    std::vector<float> w1u(size_t(np) * np, 0.f), vu(size_t(np) * np, 0.f);
    std::vector<float> w1d(size_t(np) * np, 0.f), vd(size_t(np) * np, 0.f);
    for (int r = 0; r < k; ++r)
        for (int i = 0; i < n; ++i) {
            w1u[size_t(r) * np + i] = float(U[size_t(i) * n + r] / S[r]);
            vu[size_t(i) * np + r] = float(V[size_t(i) * n + r]);
            w1d[size_t(r) * np + i] = float(V[size_t(i) * n + r] / S[r]);
            vd[size_t(i) * np + r] = float(U[size_t(i) * n + r]);
        }
    {
        std::vector<uint32_t> c(size_t(np) * np);
        frag_chain(w1u.data(), np, c.data());
        upload(op->uc2e_w1, c.data(), c.size() * 4);
        frag_chain(vu.data(), np, c.data());
        upload(op->uc2e_v, c.data(), c.size() * 4);
        frag_chain(w1d.data(), np, c.data());
        upload(op->dc2e_w1, c.data(), c.size() * 4);
        frag_chain(vd.data(), np, c.data());
        upload(op->dc2e_v, c.data(), c.size() * 4);
    }

    // M2M (parent uc <- child ue) and L2L (child dc <- parent de), parent units
    std::vector<float> m2m(size_t(8) * np * np, 0.f), l2l(size_t(8) * np * np, 0.f);
    for (int o = 0; o < 8; ++o) {
        double dlt[3] = {0.5 * (((o >> 2) & 1) - 0.5), 0.5 * (((o >> 1) & 1) - 0.5), 0.5 * ((o & 1) - 0.5)};
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double ce[3], cc[3];
                for (int d = 0; d < 3; ++d) {
                    ce[d] = dlt[d] + 0.5 * sin[3 * j + d];      // child ue
                    cc[d] = dlt[d] + 0.5 * sin[3 * i + d];      // child dc
                }
                m2m[(size_t(o) * np + i) * np + j] = float(inv_dist(&sout[3 * i], ce));
                l2l[(size_t(o) * np + i) * np + j] = float(0.5 * inv_dist(cc, &sout[3 * j]));
            }
    }
    {
        const size_t per = size_t(np) * np;
        std::vector<uint32_t> fm(8 * per), fl(8 * per);
        for (int o = 0; o < 8; ++o) {
            frag_f32(&m2m[o * per], np, &fm[o * per]);
            frag_f32(&l2l[o * per], np, &fl[o * per]);
        }
        upload(op->m2m, fm.data(), fm.size() * 4);
        upload(op->l2l, fl.data(), fl.size() * 4);
    }

    // M2L for the 316 far offsets, lexicographic (dx, dy, dz)
    std::vector<float> m2l(size_t(kNumV) * np * np, 0.f);
    std::vector<uint16_t> hi(size_t(kNumV) * np * np, 0), lo(size_t(kNumV) * np * np, 0);
    int m = 0;
    for (int dx = -3; dx <= 3; ++dx)
        for (int dy = -3; dy <= 3; ++dy)
            for (int dz = -3; dz <= 3; ++dz) {
                if (std::max(abs(dx), std::max(abs(dy), abs(dz))) <= 1) continue;
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        double src[3] = {dx + sin[3 * j], dy + sin[3 * j + 1], dz + sin[3 * j + 2]};
                        double v = inv_dist(&sin[3 * i], src);
                        size_t at = (size_t(m) * np + i) * np + j;
                        m2l[at] = float(v);
                        uint16_t h = bf16_rne(float(v));
                        hi[at] = h;
                        lo[at] = bf16_rne(float(v - double(bf16_to_float(h))));
                    }
                ++m;
            }
    {
        const size_t per = size_t(np) * np;
        std::vector<uint32_t> f32(size_t(kNumV) * per);
        std::vector<uint16_t> f16(size_t(kNumV) * per * 2);
        for (int mm = 0; mm < kNumV; ++mm) {
            frag_f32(&m2l[mm * per], np, &f32[mm * per]);
            frag_bf16(&hi[mm * per], &lo[mm * per], np, &f16[mm * per * 2]);
        }
        upload(op->m2l_f32, f32.data(), f32.size() * 4);
        upload(op->m2l_bf16, f16.data(), f16.size() * 2);
    }
    return op;
}

// Harmonic lattice kernel of a unit cell (V = 1) for a unit charge: the
// Ewald Green's function with the images |n|_inf <= 1 removed and without its
// non-harmonic part 2 pi |r|^2 / 3,
//   F(r) = sum_{|n|_inf >= 2} erfc(a R)/R - sum_{|n|_inf <= 1} erf(a R)/R
//        + 8 pi sum_{k in a half space} exp(-k^2 / (4 a^2)) / k^2 cos(k . r)
//        - pi / a^2 - 2 pi |r|^2 / 3,       R = |r + n|, k = 2 pi m,
// for all (i, j) pairs of the surface points x_i - y_j.  The splitting a = 4
// makes both sums converge below 1e-16 with |n|_inf <= 3 and |m|_inf <= 9 for
// |r|_inf <= 1.05.  The reciprocal sum factorises over the two point sets.
std::vector<double> lattice_kernel(const std::vector<double>& xs, const std::vector<double>& ys, int n) {
    const double a = 4.0;
    const int nimg = 3, mmax = 9;
    std::vector<double> F(size_t(n) * n, 0.0);
    const double c0 = 2.0 * a / sqrt(M_PI);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double r[3] = {xs[3 * i] - ys[3 * j], xs[3 * i + 1] - ys[3 * j + 1], xs[3 * i + 2] - ys[3 * j + 2]};
            double acc = 0.0;
            for (int nx = -nimg; nx <= nimg; ++nx)
                for (int ny = -nimg; ny <= nimg; ++ny)
                    for (int nz = -nimg; nz <= nimg; ++nz) {
                        const double dx = r[0] + nx, dy = r[1] + ny, dz = r[2] + nz;
                        const double R = sqrt(dx * dx + dy * dy + dz * dz);
                        const bool nearimg = std::max(abs(nx), std::max(abs(ny), abs(nz))) <= 1;
                        if (nearimg) acc -= R > 0.0 ? erf(a * R) / R : c0;
                        else acc += erfc(a * R) / R;
                    }
            F[size_t(i) * n + j] = acc - M_PI / (a * a) -
                                   2.0 * M_PI / 3.0 * (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        }
    // reciprocal part: cos(k.(x - y)) = cos(k.x) cos(k.y) + sin(k.x) sin(k.y)
    std::vector<double> wk, cx, sx, cy, sy;
    for (int mx = 0; mx <= mmax; ++mx)
        for (int my = -mmax; my <= mmax; ++my)
            for (int mz = -mmax; mz <= mmax; ++mz) {
                if (mx == 0 && (my < 0 || (my == 0 && mz <= 0))) continue;   // one of each +-m, m != 0
                const double kx = 2 * M_PI * mx, ky = 2 * M_PI * my, kz = 2 * M_PI * mz;
                const double k2 = kx * kx + ky * ky + kz * kz;
                wk.push_back(8.0 * M_PI * exp(-k2 / (4.0 * a * a)) / k2);
                for (int i = 0; i < n; ++i) {
                    const double px = kx * xs[3 * i] + ky * xs[3 * i + 1] + kz * xs[3 * i + 2];
                    const double py = kx * ys[3 * i] + ky * ys[3 * i + 1] + kz * ys[3 * i + 2];
                    cx.push_back(cos(px));
                    sx.push_back(sin(px));
                    cy.push_back(cos(py));
                    sy.push_back(sin(py));
                }
            }
    const size_t K = wk.size();
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (size_t k = 0; k < K; ++k)
                acc += wk[k] * (cx[k * n + i] * cy[k * n + j] + sx[k * n + i] * sy[k * n + j]);
            F[size_t(i) * n + j] += acc;
        }
    return F;
}

}  // namespace

namespace {

// Tile sizes the M2L kernel is instantiated for.
int m2l_tile(int k) {
    for (int t : {32, 64, 128, 160, 224, 320})
        if (t >= k) return t;
    return 0;
}

std::unique_ptr<M2LBasis> build_m2l_basis(int p, double rtol) {
    auto b = std::make_unique<M2LBasis>();
    const int n = 6 * (p - 1) * (p - 1) + 2;
    const int np = (n + 31) / 32 * 32;
    std::vector<double> sin = unit_surface(p, 1.05);
    // the 316 unit M2L operators (dc <- ue at offset d) and G = sum_d M M^T,
    // whose eigenvectors are the left singular vectors of [M(d_1) ... M(d_316)]
    std::vector<std::vector<double>> M;
    std::vector<double> G(size_t(n) * n, 0.0);
    for (int dx = -3; dx <= 3; ++dx)
        for (int dy = -3; dy <= 3; ++dy)
            for (int dz = -3; dz <= 3; ++dz) {
                if (std::max(abs(dx), std::max(abs(dy), abs(dz))) <= 1) continue;
                std::vector<double> A(size_t(n) * n);
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        double src[3] = {dx + sin[3 * j], dy + sin[3 * j + 1], dz + sin[3 * j + 2]};
                        A[size_t(i) * n + j] = inv_dist(&sin[3 * i], src);
                    }
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j <= i; ++j) {
                        double acc = 0.0;
                        for (int c = 0; c < n; ++c) acc += A[size_t(i) * n + c] * A[size_t(j) * n + c];
                        G[size_t(i) * n + j] += acc;
                    }
                M.push_back(std::move(A));
            }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) G[size_t(i) * n + j] = G[size_t(j) * n + i];
    std::vector<double> U(size_t(n) * n), S(n), V(size_t(n) * n);
    jacobi_svd(n, G.data(), U.data(), S.data(), V.data());
    // sigma_i(H) = sqrt(S_i): keep sigma_i >= rtol sigma_1
    int k = 0;
    while (k < n && S[k] >= rtol * rtol * S[0]) ++k;
    b->k = k;
    b->sigma.resize(n);
    for (int i = 0; i < n; ++i) b->sigma[i] = std::sqrt(std::max(S[i], 0.0));
    const int kp = m2l_tile(k);
    if (kp == 0 || kp >= np) return b;   // no smaller tile: the exact operators are used
    b->kp = kp;
    std::vector<float> q(size_t(np) * kp, 0.f), qt(size_t(kp) * np, 0.f);
    for (int c = 0; c < n; ++c)
        for (int r = 0; r < k; ++r) {
            q[size_t(c) * kp + r] = float(U[size_t(c) * n + r]);
            qt[size_t(r) * np + c] = float(U[size_t(c) * n + r]);
        }
    upload(b->q, q.data(), q.size() * 4);
    upload(b->qt, qt.data(), qt.size() * 4);
    // cores Q^T M(d) Q in the M2L kernel's gather-fragment order at kp
    const size_t per = size_t(kp) * kp;
    std::vector<float> core(size_t(kNumV) * per, 0.f);
    std::vector<uint16_t> hi(size_t(kNumV) * per, 0), lo(size_t(kNumV) * per, 0);
    std::vector<double> T(size_t(n) * k);
    for (int m = 0; m < kNumV; ++m) {
        const std::vector<double>& A = M[m];
        for (int i = 0; i < n; ++i)   // T = M Q
            for (int r = 0; r < k; ++r) {
                double acc = 0.0;
                for (int c = 0; c < n; ++c) acc += A[size_t(i) * n + c] * U[size_t(c) * n + r];
                T[size_t(i) * k + r] = acc;
            }
        for (int a = 0; a < k; ++a)   // Q^T T
            for (int r = 0; r < k; ++r) {
                double acc = 0.0;
                for (int i = 0; i < n; ++i) acc += U[size_t(i) * n + a] * T[size_t(i) * k + r];
                const size_t at = size_t(m) * per + size_t(a) * kp + r;
                core[at] = float(acc);
                const uint16_t h = bf16_rne(float(acc));
                hi[at] = h;
                lo[at] = bf16_rne(float(acc - double(bf16_to_float(h))));
            }
    }
    std::vector<uint32_t> f32(size_t(kNumV) * per);
    std::vector<uint16_t> f16(size_t(kNumV) * per * 2);
    for (int m = 0; m < kNumV; ++m) {
        frag_f32(&core[m * per], kp, &f32[m * per]);
        frag_bf16(&hi[m * per], &lo[m * per], kp, &f16[m * per * 2]);
    }
    upload(b->core_f32, f32.data(), f32.size() * 4);
    upload(b->core_bf16, f16.data(), f16.size() * 2);
    return b;
}

}  // namespace

const M2LBasis& get_m2l_basis(int p, double tau, double rtol) {
    static std::mutex mu;
    static auto* cache = new std::map<std::tuple<int, int, double>, std::unique_ptr<M2LBasis>>();
    (void)tau;   // the basis depends on the M2L operators only
    int dev = 0;
    KIFMM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(mu);
    auto key = std::make_tuple(dev, p, rtol);
    auto it = cache->find(key);
    if (it == cache->end()) it = cache->emplace(key, build_m2l_basis(p, rtol)).first;
    return *it->second;
}

const DBuf& get_lattice_operator(int p, double tau) {
    static std::mutex mu;
    static auto* cache = new std::map<std::tuple<int, int, double>, std::unique_ptr<DBuf>>();
    const Operators& op = get_operators(p, tau);
    int dev = 0;
    KIFMM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(mu);
    auto key = std::make_tuple(dev, p, tau);
    auto it = cache->find(key);
    if (it != cache->end()) return *it->second;
    const int n = op.n, k = op.rank;
    // the root's downward check surface is its upward equivalent surface (rho = 1.05)
    std::vector<double> srf = unit_surface(p, 1.05);
    std::vector<double> T = lattice_kernel(srf, srf, n);
    // DC2E = U Sigma^-1 V^T (truncated): R = U (Sigma^-1 (V^T T))
    std::vector<double> W(size_t(k) * n, 0.0), R(size_t(n) * n, 0.0);
    for (int r = 0; r < k; ++r)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int l = 0; l < n; ++l) acc += op.svd_v[size_t(l) * n + r] * T[size_t(l) * n + j];
            W[size_t(r) * n + j] = acc / op.sigma[r];
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int r = 0; r < k; ++r) acc += op.svd_u[size_t(i) * n + r] * W[size_t(r) * n + j];
            R[size_t(i) * n + j] = acc;
        }
    auto buf = std::make_unique<DBuf>();
    upload(*buf, R.data(), R.size() * sizeof(double));
    it = cache->emplace(key, std::move(buf)).first;
    return *it->second;
}

const Operators& get_operators(int p, double tau) {
    // Kept until the process ends (never destroyed: the HIP runtime may be gone
    // by the time static destructors run).
    static std::mutex mu;
    static auto* cache = new std::map<std::tuple<int, int, double>, std::unique_ptr<Operators>>();
    int dev = 0;
    KIFMM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(mu);
    auto key = std::make_tuple(dev, p, tau);
    auto it = cache->find(key);
    if (it == cache->end()) it = cache->emplace(key, build_operators(p, tau)).first;
    return *it->second;
}

}  // namespace kifmm
