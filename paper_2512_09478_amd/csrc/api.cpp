// C ABI of the library: argument checks, plan lifetime and the order of the
// kernel launches of one evaluation (Section 2.2: tree, upward pass, downward
// pass, leaf evaluation), its transposed sweep, and the clump aggregation of
// Section 2.4.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>

#include "common.h"

using namespace kifmm;

namespace {

thread_local std::string g_err;

template <class F>
int guarded(F&& f) {
    try {
        f();
        return KIFMM_OK;
    } catch (const Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return KIFMM_ERR_OOM;
    } catch (const std::exception& e) {
        g_err = e.what();
        return KIFMM_ERR_STATE;
    }
}

void check_options(const kifmm_options& o) {
    if (o.max_depth < 0 || o.max_depth > kBits) throw Error(KIFMM_ERR_ARG, "max_depth must be in 0..21");
    if (o.precision != KIFMM_FP32 && o.precision != KIFMM_SPLIT_BF16) throw Error(KIFMM_ERR_ARG, "unknown precision");
    if (!(o.pinv_rtol > 0.0 && o.pinv_rtol < 1.0)) throw Error(KIFMM_ERR_ARG, "pinv_rtol must be in (0, 1)");
    if (o.periodic && !o.explicit_root) throw Error(KIFMM_ERR_ARG, "a periodic plan needs the cell as an explicit root");
    if (!(o.m2l_rtol >= 0.0 && o.m2l_rtol < 1.0)) throw Error(KIFMM_ERR_ARG, "m2l_rtol must be in [0, 1)");
    if (o.explicit_root) {
        int e = 0;
        double m = frexp(o.root_side, &e);
        if (!(o.root_side > 0.0) || m != 0.5) throw Error(KIFMM_ERR_ARG, "root_side must be a power of two");
        for (int d = 0; d < 3; ++d) {
            double g = o.root_lo[d] * 4096.0 / o.root_side;
            if (!isfinite(g) || g != floor(g)) throw Error(KIFMM_ERR_ARG, "root_lo must lie on the root_side/4096 grid");
        }
    }
}

void alloc_densities(kifmm_plan* P, hipStream_t s) {
    size_t bytes = size_t(2) * size_t(P->B) * P->npad * 4;
    for (DBuf* b : {&P->psi_u, &P->phi_u, &P->psi_d, &P->phi_d}) {
        bool fresh = b->cap < bytes;
        b->ensure(bytes);
        if (fresh) KIFMM_HIP(hipMemsetAsync(b->p, 0, b->cap, s));
    }
    // small trees get more M2L partial buffers (see launch_m2l)
    P->m2l_split_cap = bytes <= (size_t(64) << 20) ? kM2LSplitMax : kM2LSplit;
    P->psi_m.ensure(size_t(P->m2l_split_cap) * bytes);
    if (P->cm) P->phi_k.ensure(size_t(2) * size_t(P->B) * P->cm->kp * 4);
    P->nearv.ensure(size_t(P->N) * 16);
    if (P->periodic) {
        P->mom.ensure(2 * 16 * sizeof(double));
        P->mom_part.ensure(size_t(kMomentBlocks) * 16 * sizeof(double));
    }
}

kifmm_plan* checked(kifmm_handle h) {
    if (!h) throw Error(KIFMM_ERR_STATE, "null handle");
    if (h->B <= 0) throw Error(KIFMM_ERR_STATE, "handle has no tree");
    return h;
}

void begin_phases(kifmm_plan* P, hipStream_t s) {
    if (!P->opt.profile) return;
    PhaseEvents& pe = P->events;
    if (!pe.made) {
        for (auto& row : pe.ev)
            for (auto& e : row) KIFMM_HIP(hipEventCreate(&e));
        for (auto& row : pe.p2p)
            for (auto& e : row) KIFMM_HIP(hipEventCreate(&e));
        pe.made = true;
    }
    pe.cur = (pe.cur + 1) % PhaseEvents::kRing;
    pe.valid[pe.cur] = false;
    ++pe.calls;
    KIFMM_HIP(hipEventRecord(pe.ev[pe.cur][0], s));
}

// the profiled call has recorded all its events
void end_phases(kifmm_plan* P) {
    if (P->opt.profile && P->events.made) P->events.valid[P->events.cur] = true;
}

enum NearKind { NEAR_FORWARD, NEAR_BACKWARD, NEAR_DIPOLES, NEAR_GRAD, NEAR_GRAD_DIPOLES, NEAR_FORWARD_EXCL,
                NEAR_BACKWARD_EXCL, NEAR_STOKES };

// The near field does not depend on the far-field sweep: it runs on the side
// stream, forked from `s` after P2M (so that the sweep's first kernel is not
// queued behind it) and joined back before the leaf evaluation, which adds it
// to the far field.
void fork_near(kifmm_plan* P, NearKind kind, hipStream_t s, double viscosity = 1.0) {
    P->nearq.make();
    hipStream_t t = P->nearq.s;
    KIFMM_HIP(hipEventRecord(P->nearq.fork, s));
    KIFMM_HIP(hipStreamWaitEvent(t, P->nearq.fork, 0));
    const bool prof = P->opt.profile && P->events.made;
    if (prof) KIFMM_HIP(hipEventRecord(P->events.p2p[P->events.cur][0], t));
    if (kind == NEAR_BACKWARD || kind == NEAR_BACKWARD_EXCL) launch_p2p_backward(P, t, kind == NEAR_BACKWARD_EXCL);
    else if (kind == NEAR_DIPOLES) launch_p2p_dipoles(P, t);
    else if (kind == NEAR_STOKES) launch_p2p_stokes(P, viscosity, t);
    else if (kind == NEAR_GRAD || kind == NEAR_GRAD_DIPOLES) launch_p2p_gradient(P, kind == NEAR_GRAD_DIPOLES, t);
    else launch_p2p_forward(P, t, kind == NEAR_FORWARD_EXCL);
    if (prof) KIFMM_HIP(hipEventRecord(P->events.p2p[P->events.cur][1], t));
    KIFMM_HIP(hipEventRecord(P->nearq.join, t));
}

void join_near(kifmm_plan* P, hipStream_t s) {
    KIFMM_HIP(hipStreamWaitEvent(s, P->nearq.join, 0));
    record_phase(P, 5, s);
}

}  // namespace

namespace kifmm {
void record_phase(kifmm_plan* P, int idx, hipStream_t s) {
    if (!P->opt.profile || !P->events.made) return;
    KIFMM_HIP(hipEventRecord(P->events.ev[P->events.cur][idx + 1], s));
}
}  // namespace kifmm

extern "C" {

void kifmm_default_options(kifmm_options* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->adaptive = 1;
    o->max_depth = kBits;
    o->precision = KIFMM_FP32;
    o->pinv_rtol = 1e-7;
    o->explicit_root = 0;
    o->root_side = 1.0;
    o->profile = 0;
}

int kifmm_setup_ex(const double* positions, int64_t N, int kernel, int p, int leaf_size, const kifmm_options* opts,
                   void* stream, kifmm_handle* out) {
    kifmm_plan* P = nullptr;
    int rc = guarded([&] {
        if (!out) throw Error(KIFMM_ERR_ARG, "null output handle pointer");
        *out = nullptr;
        if (!positions) throw Error(KIFMM_ERR_ARG, "null positions");
        if (N < 1 || N >= (int64_t(1) << 31)) throw Error(KIFMM_ERR_ARG, "N must be in 1..2^31-1");
        if (kernel != KIFMM_LAPLACE && kernel != KIFMM_GRAVITY) throw Error(KIFMM_ERR_ARG, "unknown kernel");
        if (opts && opts->periodic && kernel != KIFMM_LAPLACE)
            throw Error(KIFMM_ERR_ARG, "periodic sums are defined for the Laplace kernel only");
        if (p < 2 || p > 8) throw Error(KIFMM_ERR_ARG, "p must be in 2..8");
        if (leaf_size < 1) throw Error(KIFMM_ERR_ARG, "leaf_size must be >= 1");
        kifmm_options o;
        kifmm_default_options(&o);
        if (opts) o = *opts;
        check_options(o);
        hipStream_t s = static_cast<hipStream_t>(stream);
        P = new kifmm_plan();
        P->kernel = kernel;
        P->c = kernel == KIFMM_LAPLACE ? 1.0 / (4.0 * M_PI) : -1.0;
        P->p = p;
        P->leaf = leaf_size;
        P->opt = o;
        P->N = N;
        P->periodic = o.periodic != 0;
        P->ops = &get_operators(p, o.pinv_rtol);
        if (o.m2l_rtol > 0.0) {
            const M2LBasis& cm = get_m2l_basis(p, o.pinv_rtol, o.m2l_rtol);
            if (cm.kp > 0) P->cm = &cm;
        }
        if (P->periodic) (void)get_lattice_operator(p, o.pinv_rtol);
        P->n = P->ops->n;
        P->npad = P->ops->npad;
        P->last_stream = s;
        P->status.ensure(sizeof(int));
        KIFMM_HIP(hipMemsetAsync(P->status.p, 0, sizeof(int), s));
        (void)noalloc_scratch();   // the fixed scratch's address on this device
        build_tree(P, positions, s);
        alloc_densities(P, s);
        KIFMM_HIP(hipStreamSynchronize(s));
        *out = P;
    });
    if (rc != KIFMM_OK && P) {
        delete P;
        if (out) *out = nullptr;
    }
    return rc;
}

int kifmm_setup(const double* positions, int64_t N, int kernel, int p, int leaf_size, kifmm_handle* out) {
    return kifmm_setup_ex(positions, N, kernel, p, leaf_size, nullptr, nullptr, out);
}

int kifmm_rebuild(kifmm_handle h, const double* positions, void* stream) {
    return guarded([&] {
        if (!h) throw Error(KIFMM_ERR_STATE, "null handle");
        if (!positions) throw Error(KIFMM_ERR_ARG, "null positions");
        hipStream_t s = static_cast<hipStream_t>(stream);
        h->last_stream = s;
        h->B = 0;
        h->fwd_valid = false;
        h->fwd_excl = false;
        build_tree(h, positions, s);
        alloc_densities(h, s);
        launch_clump_ids(h, s);
        KIFMM_HIP(hipStreamSynchronize(s));
    });
}

int kifmm_set_precision(kifmm_handle h, int precision) {
    return guarded([&] {
        if (!h) throw Error(KIFMM_ERR_STATE, "null handle");
        if (precision != KIFMM_FP32 && precision != KIFMM_SPLIT_BF16) throw Error(KIFMM_ERR_ARG, "unknown precision");
        h->opt.precision = precision;
        h->fwd_valid = false;
        h->fwd_excl = false;
    });
}

int kifmm_evaluate(kifmm_handle h, const float* charges, float* potential, float* field, void* stream) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (!charges) throw Error(KIFMM_ERR_ARG, "null charges");
        hipStream_t s = static_cast<hipStream_t>(stream);
        P->last_stream = s;
        begin_phases(P, s);
        P->fwd_valid = false;
        P->fwd_excl = false;
        launch_gather(P, charges, nullptr, nullptr, false, s);
        run_sweep(P, 0, 1, s, true, [&] { fork_near(P, NEAR_FORWARD, s); });
        join_near(P, s);
        run_far_eval(P, false, potential, field, s);
        record_phase(P, 6, s);
        end_phases(P);
        P->fwd_valid = true;
        KIFMM_HIP(hipGetLastError());
    });
}

int kifmm_evaluate_dipoles(kifmm_handle h, const float* charges, const float* dipoles, float* potential,
                           float* field, void* stream) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (!dipoles) throw Error(KIFMM_ERR_ARG, "null dipoles");
        hipStream_t s = static_cast<hipStream_t>(stream);
        P->last_stream = s;
        begin_phases(P, s);
        // the sources go through the adjoint right-hand side (1): monopoles and
        // dipoles; the sorted points' charges are overwritten, so a later
        // kifmm_backward must pass its charges
        P->fwd_valid = false;
        P->fwd_excl = false;
        launch_gather(P, charges, charges, dipoles, true, s, true);
        run_sweep(P, 1, 2, s, true, [&] { fork_near(P, NEAR_DIPOLES, s); });
        join_near(P, s);
        run_far_eval(P, false, potential, field, s, 1);
        record_phase(P, 6, s);
        end_phases(P);
        KIFMM_HIP(hipGetLastError());
    });
}

int kifmm_evaluate_gradient(kifmm_handle h, const float* charges, const float* dipoles, float* potential,
                            float* field, float* field_grad, void* stream) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (!charges && !dipoles) throw Error(KIFMM_ERR_ARG, "null charges and dipoles");
        hipStream_t s = static_cast<hipStream_t>(stream);
        P->last_stream = s;
        begin_phases(P, s);
        P->fwd_valid = false;
        P->fwd_excl = false;
        // with dipoles the sources go through right-hand side 1 (as in
        // kifmm_evaluate_dipoles), otherwise through 0
        const int rhs = dipoles ? 1 : 0;
        launch_gather(P, charges, charges, dipoles, dipoles != nullptr, s, true);
        run_sweep(P, rhs, rhs + 1, s, true,
                  [&] { fork_near(P, dipoles ? NEAR_GRAD_DIPOLES : NEAR_GRAD, s); });
        join_near(P, s);
        run_far_grad(P, potential, field, field_grad, s, rhs);
        record_phase(P, 6, s);
        end_phases(P);
        KIFMM_HIP(hipGetLastError());
    });
}

int kifmm_evaluate_stokes(kifmm_handle h, const float* forces, double viscosity, float* velocity, void* stream) {
    return kifmm_evaluate_stokes_ex(h, forces, viscosity, velocity, nullptr, stream);
}

int kifmm_evaluate_stokes_ex(kifmm_handle h, const float* forces, double viscosity, float* velocity, float* pressure,
                             void* stream) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (!forces || !velocity) throw Error(KIFMM_ERR_ARG, "null forces or velocity");
        if (!(viscosity > 0.0) || !std::isfinite(viscosity)) throw Error(KIFMM_ERR_ARG, "viscosity must be positive");
        if (P->kernel != KIFMM_LAPLACE) throw Error(KIFMM_ERR_STATE, "Stokes sums need a Laplace plan");
        if (P->periodic) throw Error(KIFMM_ERR_STATE, "Stokes sums are free-space only");
        hipStream_t s = static_cast<hipStream_t>(stream);
        P->last_stream = s;
        begin_phases(P, s);
        P->fwd_valid = false;
        P->fwd_excl = false;
        const size_t N = size_t(P->N);
        float* pot = static_cast<float*>(P->stk_far.ensure(N * 16 * sizeof(float)));
        float* fld = pot + 4 * N;
        // charges f_x, f_y: one sweep with two right-hand sides, the Stokeslet
        // near field on the side stream beside it
        launch_gather_stokes(P, forces, 0, s);
        run_sweep(P, 0, 2, s, true, [&] { fork_near(P, NEAR_STOKES, s, viscosity); });
        for (int r = 0; r < 2; ++r)
            run_far_eval(P, false, pot + r * N, fld + 3 * r * N, s, r, false, false, nullptr, true);
        // the first sweep's upward, compressed and downward densities of f_x
        // and f_y, which the second sweep's framed charge needs after the
        // second sweep has overwritten them
        const size_t sU = size_t(P->B) * P->npad, sK = P->cm ? size_t(P->B) * P->cm->kp : 0;
        float* keep = static_cast<float*>(P->stk_keep.ensure((4 * sU + 2 * sK) * sizeof(float)));
        float* keep_u = keep;
        float* keep_d = keep + 2 * sU;
        float* keep_k = keep + 4 * sU;
        KIFMM_HIP(hipMemcpyAsync(keep_u, P->phi_u.p, 2 * sU * sizeof(float), hipMemcpyDeviceToDevice, s));
        KIFMM_HIP(hipMemcpyAsync(keep_d, P->phi_d.p, 2 * sU * sizeof(float), hipMemcpyDeviceToDevice, s));
        if (sK) KIFMM_HIP(hipMemcpyAsync(keep_k, P->phi_k.p, 2 * sK * sizeof(float), hipMemcpyDeviceToDevice, s));
        // charges f_z and (x - c).f about each box's centre c
        launch_gather_stokes(P, forces, 1, s);
        StokesFrames sf;
        sf.frc = P->stk.as<float4>();
        const float* cur_u = P->phi_u.as<float>();
        const float* cur_d = P->phi_d.as<float>();
        const float* cur_k = sK ? P->phi_k.as<float>() : nullptr;
        for (int k = 0; k < 2; ++k) {
            sf.up[k] = keep_u + k * sU;
            sf.dn[k] = keep_d + k * sU;
            sf.kp[k] = sK ? keep_k + k * sK : nullptr;
        }
        sf.up[2] = cur_u;   // f_z: right-hand side 0 of this sweep, done before right-hand side 1
        sf.dn[2] = cur_d;
        sf.kp[2] = cur_k;
        run_sweep(P, 0, 2, s, false, [] {}, &sf);
        run_far_eval(P, false, pot + 2 * N, fld + 3 * 2 * N, s, 0, false, false, nullptr, true);
        run_far_eval(P, false, pot + 3 * N, fld + 3 * 3 * N, s, 1, false, false, &sf, true);
        launch_stokes_frames(P, s);
        join_near(P, s);
        launch_stokes_combine(P, viscosity, velocity, pressure, s);
        record_phase(P, 6, s);
        end_phases(P);
        KIFMM_HIP(hipGetLastError());
    });
}

int kifmm_backward(kifmm_handle h, const float* charges, const float* grad_potential, const float* grad_field,
                   float* grad_charges, float* grad_positions, void* stream) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (!charges && !P->fwd_valid)
            throw Error(KIFMM_ERR_STATE, "no forward evaluation to reuse (null charges after setup, rebuild or "
                                         "a precision change)");
        hipStream_t s = static_cast<hipStream_t>(stream);
        P->last_stream = s;
        begin_phases(P, s);
        // null charges: the charges, sorted points and densities of the last
        // forward pass are still in place and only the adjoint sources are swept
        if (charges) {
            P->fwd_valid = false;
            P->fwd_excl = false;
        }
        launch_gather(P, charges, grad_potential, grad_field, true, s);
        run_sweep(P, charges ? 0 : 1, 2, s, true, [&] { fork_near(P, NEAR_BACKWARD, s); });
        P->fwd_valid = true;
        join_near(P, s);
        run_far_eval(P, true, grad_charges, grad_positions, s);
        record_phase(P, 6, s);
        end_phases(P);
        KIFMM_HIP(hipGetLastError());
    });
}

}  // extern "C"

extern "C" {

int kifmm_clump_reduce(kifmm_handle h, const float* charges, const float* field, const int64_t* clump_offsets,
                       int64_t C, const double* centers, double* force, double* torque, void* stream) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (C < 0 || C >= (int64_t(1) << 31)) throw Error(KIFMM_ERR_ARG, "clump count out of range");
        if (C == 0) return;
        if (!charges || !field || !clump_offsets || !centers || !force || !torque)
            throw Error(KIFMM_ERR_ARG, "null pointer argument");
        hipStream_t s = static_cast<hipStream_t>(stream);
        P->last_stream = s;
        P->clump_part.ensure(clump_scratch_bytes(P->N, 6));
        launch_clump_reduce(P, charges, field, clump_offsets, nullptr, C, centers, force, torque,
                            P->clump_part.as<double>(), s);
        KIFMM_HIP(hipGetLastError());
    });
}

int kifmm_clump_reduce_noalloc(kifmm_handle h, const float* charges, const float* field,
                               const int64_t* clump_offsets, int64_t C, const double* centers, double* force,
                               double* torque, void* stream) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (C < 0 || C >= (int64_t(1) << 31)) throw Error(KIFMM_ERR_ARG, "clump count out of range");
        if (clump_scratch_bytes(P->N, 6) > kNoAllocScratchBytes)
            throw Error(KIFMM_ERR_ARG, "N beyond the fixed scratch of kifmm_clump_reduce_noalloc (11,184,640 points)");
        if (C == 0) return;
        if (!charges || !field || !clump_offsets || !centers || !force || !torque)
            throw Error(KIFMM_ERR_ARG, "null pointer argument");
        hipStream_t s = static_cast<hipStream_t>(stream);
        P->last_stream = s;
        launch_clump_reduce(P, charges, field, clump_offsets, nullptr, C, centers, force, torque,
                            static_cast<double*>(noalloc_scratch()), s);
        KIFMM_HIP(hipGetLastError());
    });
}

int kifmm_clump_backward(kifmm_handle h, const float* charges, const float* field, const int64_t* clump_offsets,
                         int64_t C, const double* centers, const double* grad_force, const double* grad_torque,
                         float* grad_charges, float* grad_field, float* grad_positions, double* grad_centers,
                         void* stream) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (C < 0 || C >= (int64_t(1) << 31)) throw Error(KIFMM_ERR_ARG, "clump count out of range");
        if (!charges || !field || (C > 0 && (!clump_offsets || !centers)))
            throw Error(KIFMM_ERR_ARG, "null pointer argument");
        hipStream_t s = static_cast<hipStream_t>(stream);
        P->last_stream = s;
        P->clump_part.ensure(clump_scratch_bytes(P->N, 6));
        launch_clump_backward(P, charges, field, clump_offsets, nullptr, C, centers, grad_force, grad_torque,
                              grad_charges, grad_field, grad_positions, false, C > 0 ? grad_centers : nullptr,
                              P->clump_part.as<double>(), s);
        KIFMM_HIP(hipGetLastError());
    });
}

int kifmm_set_clumps(kifmm_handle h, const int64_t* clump_offsets, int64_t C, void* stream) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (C < 0 || C >= (int64_t(1) << 31)) throw Error(KIFMM_ERR_ARG, "clump count out of range");
        hipStream_t s = static_cast<hipStream_t>(stream);
        P->last_stream = s;
        if (P->fwd_excl) P->fwd_valid = false;
        P->fwd_excl = false;
        P->clumps = 0;
        if (C == 0) return;
        if (!clump_offsets) throw Error(KIFMM_ERR_ARG, "null clump offsets");
        std::vector<int64_t> off(size_t(C) + 1);
        KIFMM_HIP(hipMemcpyAsync(off.data(), clump_offsets, off.size() * 8, hipMemcpyDeviceToHost, s));
        KIFMM_HIP(hipStreamSynchronize(s));
        if (off[0] != 0 || off[size_t(C)] > P->N) throw Error(KIFMM_ERR_INPUT, "clump offsets out of range");
        for (int64_t c = 0; c < C; ++c)
            if (off[size_t(c) + 1] < off[size_t(c)]) throw Error(KIFMM_ERR_INPUT, "clump offsets not monotone");
        P->clump_off.ensure(off.size() * 8);
        KIFMM_HIP(hipMemcpyAsync(P->clump_off.p, off.data(), off.size() * 8, hipMemcpyHostToDevice, s));
        set_clump_ids(P, P->clump_off.as<int64_t>(), C, s);
        P->clumps = C;
        launch_clump_ids(P, s);
        P->clump_part.ensure(clump_scratch_bytes(P->N, 6));
        KIFMM_HIP(hipStreamSynchronize(s));
    });
}

int kifmm_clump_forces(kifmm_handle h, const float* charges, const double* centers, double* force, double* torque,
                       float* field, void* stream) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (P->clumps <= 0) throw Error(KIFMM_ERR_STATE, "no clumps registered (kifmm_set_clumps)");
        if (!charges || !centers || !force || !torque) throw Error(KIFMM_ERR_ARG, "null pointer argument");
        hipStream_t s = static_cast<hipStream_t>(stream);
        P->last_stream = s;
        begin_phases(P, s);
        P->fwd_valid = false;
        P->fwd_excl = false;
        launch_gather(P, charges, nullptr, nullptr, false, s);
        run_sweep(P, 0, 1, s, true, [&] { fork_near(P, NEAR_FORWARD_EXCL, s); });
        join_near(P, s);
        float* E = P->clump_E.ensure(size_t(P->N) * 12) ? P->clump_E.as<float>() : nullptr;
        run_far_eval(P, false, nullptr, E, s);
        record_phase(P, 6, s);
        launch_clump_reduce(P, charges, E, P->clump_off.as<int64_t>(), P->cid.as<int>(), P->clumps, centers, force,
                            torque, P->clump_part.as<double>(), s);
        if (field) KIFMM_HIP(hipMemcpyAsync(field, E, size_t(P->N) * 12, hipMemcpyDeviceToDevice, s));
        end_phases(P);
        P->fwd_valid = true;
        P->fwd_excl = true;
        KIFMM_HIP(hipGetLastError());
    });
}

int kifmm_clump_forces_backward(kifmm_handle h, const float* charges, const double* centers,
                                const double* grad_force, const double* grad_torque, float* grad_charges,
                                float* grad_positions, double* grad_centers, void* stream) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (!P->fwd_valid || !P->fwd_excl || P->clumps <= 0)
            throw Error(KIFMM_ERR_STATE, "no kifmm_clump_forces evaluation to differentiate");
        if (!charges || !centers) throw Error(KIFMM_ERR_ARG, "null pointer argument");
        hipStream_t s = static_cast<hipStream_t>(stream);
        P->last_stream = s;
        begin_phases(P, s);
        float* Eb = P->clump_Eb.ensure(size_t(P->N) * 12) ? P->clump_Eb.as<float>() : nullptr;
        // the aggregation's direct parts into the outputs, its dL/dE into Eb
        launch_clump_backward(P, charges, P->clump_E.as<float>(), P->clump_off.as<int64_t>(), P->cid.as<int>(),
                              P->clumps, centers, grad_force, grad_torque, grad_charges, Eb, grad_positions, false,
                              grad_centers, P->clump_part.as<double>(), s);
        // the FMM part for the dipole sources dL/dE (forward densities reused),
        // the same pairs left out, added to the outputs
        launch_gather(P, nullptr, nullptr, Eb, true, s);
        run_sweep(P, 1, 2, s, true, [&] { fork_near(P, NEAR_BACKWARD_EXCL, s); });
        join_near(P, s);
        run_far_eval(P, true, grad_charges, grad_positions, s, 0, true);
        record_phase(P, 6, s);
        end_phases(P);
        KIFMM_HIP(hipGetLastError());
    });
}

int kifmm_synchronize(kifmm_handle h, void* stream) {
    return guarded([&] {
        if (!h) throw Error(KIFMM_ERR_STATE, "null handle");
        hipStream_t s = static_cast<hipStream_t>(stream);
        unsigned long long* w = h->host.get();
        w[63] = 0;
        KIFMM_HIP(hipMemcpyAsync(&w[63], h->status.p, sizeof(int), hipMemcpyDeviceToHost, s));
        KIFMM_HIP(hipMemsetAsync(h->status.p, 0, sizeof(int), s));
        KIFMM_HIP(hipStreamSynchronize(s));
        if (static_cast<int>(w[63] & 0xffffffffull))
            throw Error(KIFMM_ERR_INPUT, "clump offsets of an earlier call were not a valid CSR (its clumps got NaN)");
    });
}

int kifmm_get_counts(kifmm_handle h, int64_t out[10]) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (!out) throw Error(KIFMM_ERR_ARG, "null output");
        if (!P->pairs_counted) count_pairs(P, P->last_stream);
        for (int k = 0; k < 10; ++k) out[k] = P->counts[k];
    });
}

int kifmm_get_build_stats(kifmm_handle h, int64_t out[3]) {
    return guarded([&] {
        if (!h) throw Error(KIFMM_ERR_STATE, "null handle");
        if (!out) throw Error(KIFMM_ERR_ARG, "null output");
        out[0] = h->builds;
        out[1] = h->resort_steps;
        out[2] = h->resort_hits;
    });
}

int kifmm_get_m2l_rank(kifmm_handle h, int64_t out[2]) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (!out) throw Error(KIFMM_ERR_ARG, "null output");
        out[0] = P->cm ? P->cm->k : P->n;
        out[1] = P->cm ? P->cm->kp : P->npad;
    });
}

int kifmm_get_operator(kifmm_handle h, int which, double* values, int64_t cap, int64_t out[2]) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (!out) throw Error(KIFMM_ERR_ARG, "null output");
        const Operators& op = *P->ops;
        const int n = op.n;
        std::vector<double> v;
        if (which == 0) {
            v = op.sigma;
            out[1] = op.rank;
        } else if (which == 1) {
            if (!(P->opt.m2l_rtol > 0.0)) throw Error(KIFMM_ERR_STATE, "the plan has no M2L basis (m2l_rtol = 0)");
            const M2LBasis& cm = get_m2l_basis(P->p, P->opt.pinv_rtol, P->opt.m2l_rtol);
            v = cm.sigma;
            out[1] = cm.k;
        } else if (which == 2) {
            // UC2E = V_k diag(1 / sigma_k) U_k^T, unit box, kernel 1/r
            v.assign(size_t(n) * n, 0.0);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    double acc = 0.0;
                    for (int r = 0; r < op.rank; ++r)
                        acc += op.svd_v[size_t(i) * n + r] / op.sigma[r] * op.svd_u[size_t(j) * n + r];
                    v[size_t(i) * n + j] = acc;
                }
            out[1] = op.rank;
        } else {
            throw Error(KIFMM_ERR_ARG, "which must be 0, 1 or 2");
        }
        out[0] = int64_t(v.size());
        if (values) {
            if (cap < int64_t(v.size())) throw Error(KIFMM_ERR_ARG, "values buffer too small");
            std::copy(v.begin(), v.end(), values);
        }
    });
}

int kifmm_copy_tree(kifmm_handle h, uint64_t* keys, int64_t* perm, int32_t* level, int32_t* anchor, int64_t* begin,
                    int64_t* end, int64_t* parent, int8_t* is_leaf, double* root) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        hipStream_t s = P->last_stream;
        KIFMM_HIP(hipStreamSynchronize(s));
        const int64_t N = P->N, B = P->B;
        if (keys) KIFMM_HIP(hipMemcpy(keys, P->keys.p, size_t(N) * 8, hipMemcpyDeviceToHost));
        if (perm) {
            std::vector<int> t(static_cast<size_t>(N));
            KIFMM_HIP(hipMemcpy(t.data(), P->perm.p, size_t(N) * 4, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < N; ++i) perm[i] = t[size_t(i)];
        }
        if (level || anchor) {
            std::vector<int4> a(static_cast<size_t>(B));
            KIFMM_HIP(hipMemcpy(a.data(), P->bx_anchor.p, size_t(B) * 16, hipMemcpyDeviceToHost));
            for (int64_t b = 0; b < B; ++b) {
                if (level) level[b] = a[size_t(b)].w;
                if (anchor) {
                    anchor[3 * b] = a[size_t(b)].x;
                    anchor[3 * b + 1] = a[size_t(b)].y;
                    anchor[3 * b + 2] = a[size_t(b)].z;
                }
            }
        }
        if (begin || end) {
            std::vector<int2> r(static_cast<size_t>(B));
            KIFMM_HIP(hipMemcpy(r.data(), P->bx_range.p, size_t(B) * 8, hipMemcpyDeviceToHost));
            for (int64_t b = 0; b < B; ++b) {
                if (begin) begin[b] = r[size_t(b)].x;
                if (end) end[b] = r[size_t(b)].y;
            }
        }
        if (parent) {
            std::vector<int> t(static_cast<size_t>(B));
            KIFMM_HIP(hipMemcpy(t.data(), P->bx_parent.p, size_t(B) * 4, hipMemcpyDeviceToHost));
            for (int64_t b = 0; b < B; ++b) parent[b] = t[size_t(b)];
        }
        if (is_leaf) {
            std::vector<int> t(static_cast<size_t>(B));
            KIFMM_HIP(hipMemcpy(t.data(), P->bx_leaf.p, size_t(B) * 4, hipMemcpyDeviceToHost));
            for (int64_t b = 0; b < B; ++b) is_leaf[b] = int8_t(t[size_t(b)]);
        }
        if (root) {
            root[0] = P->lo[0];
            root[1] = P->lo[1];
            root[2] = P->lo[2];
            root[3] = P->side;
        }
    });
}

int kifmm_copy_list(kifmm_handle h, char which, int64_t* offsets, int64_t* indices) {
    return guarded([&] {
        kifmm_plan* P = checked(h);
        if (!offsets) throw Error(KIFMM_ERR_ARG, "null offsets");
        KIFMM_HIP(hipStreamSynchronize(P->last_stream));
        const int64_t B = P->B;
        std::vector<int> off(size_t(B) + 1), idx;
        if (which == 'U' || which == 'W' || which == 'X' || which == 'N') {
            const DBuf& o = which == 'U' ? P->u_off : which == 'W' ? P->w_off : which == 'X' ? P->x_off : P->n_off;
            const DBuf& ix = which == 'U' ? P->u_idx : which == 'W' ? P->w_idx : which == 'X' ? P->x_idx : P->n_idx;
            KIFMM_HIP(hipMemcpy(off.data(), o.p, off.size() * 4, hipMemcpyDeviceToHost));
            idx.resize(size_t(off[size_t(B)]));
            if (!idx.empty()) KIFMM_HIP(hipMemcpy(idx.data(), ix.p, idx.size() * 4, hipMemcpyDeviceToHost));
        } else if (which == 'V') {
            const int64_t b2 = P->bfar;
            std::vector<int> vd(size_t(B - b2) * kVPerOct);
            if (!vd.empty()) KIFMM_HIP(hipMemcpy(vd.data(), P->vdense.p, vd.size() * 4, hipMemcpyDeviceToHost));
            std::vector<int4> anc;
            if (P->periodic) {
                anc.resize(size_t(B));
                KIFMM_HIP(hipMemcpy(anc.data(), P->bx_anchor.p, anc.size() * sizeof(int4), hipMemcpyDeviceToHost));
            }
            off[0] = 0;
            for (int64_t b = 0; b < B; ++b) {
                if (b >= b2) {
                    size_t at = idx.size();
                    for (int j = 0; j < kVPerOct; ++j) {
                        int v = vd[size_t(b - b2) * kVPerOct + j];
                        if (v < 0) continue;
                        if (P->periodic) {
                            // the slot's cell a + d wraps around the root: record the image shift
                            const int4 a = anc[size_t(b)];
                            const int o = ((a.x & 1) << 2) | ((a.y & 1) << 1) | (a.z & 1);
                            int d[3];
                            v_slot_offset(o, j, d);
                            const int lim = 1 << a.w;
                            const int g[3] = {a.x + d[0], a.y + d[1], a.z + d[2]};
                            int sh[3];
                            for (int k = 0; k < 3; ++k) sh[k] = g[k] < 0 ? -1 : (g[k] >= lim ? 1 : 0);
                            v = img_encode(v, sh[0], sh[1], sh[2]);
                        }
                        idx.push_back(v);
                    }
                    std::sort(idx.begin() + at, idx.end());
                }
                off[size_t(b) + 1] = int(idx.size());
            }
        } else {
            throw Error(KIFMM_ERR_ARG, "list must be one of U, V, W, X, N");
        }
        for (int64_t b = 0; b <= B; ++b) offsets[b] = off[size_t(b)];
        if (indices)
            for (size_t k = 0; k < idx.size(); ++k) indices[k] = idx[k];
    });
}

int kifmm_get_phase_times_at(kifmm_handle h, int back, float* out, int n) {
    int written = 0;
    int rc = guarded([&] {
        kifmm_plan* P = checked(h);
        if (!out) throw Error(KIFMM_ERR_ARG, "null output");
        const PhaseEvents& pe = P->events;
        if (!pe.made) return;
        if (back < 0 || back >= PhaseEvents::kRing || back >= pe.calls)
            throw Error(KIFMM_ERR_ARG, "no profiled call that far back");
        const int k = ((pe.cur - back) % PhaseEvents::kRing + PhaseEvents::kRing) % PhaseEvents::kRing;
        if (!pe.valid[k]) return;
        const hipEvent_t* ev = pe.ev[k];
        KIFMM_HIP(hipEventSynchronize(ev[7]));
        KIFMM_HIP(hipEventSynchronize(pe.p2p[k][1]));
        float ms[8] = {};
        for (int i = 0; i < 5; ++i) KIFMM_HIP(hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]));
        KIFMM_HIP(hipEventElapsedTime(&ms[5], ev[6], ev[7]));
        KIFMM_HIP(hipEventElapsedTime(&ms[6], pe.p2p[k][0], pe.p2p[k][1]));
        KIFMM_HIP(hipEventElapsedTime(&ms[7], ev[0], ev[7]));
        for (int i = 0; i < std::min(n, 8); ++i) out[i] = ms[i];
        written = std::min(n, 8);
    });
    return rc == KIFMM_OK ? written : rc;
}

int kifmm_get_phase_times(kifmm_handle h, float* out, int n) { return kifmm_get_phase_times_at(h, 0, out, n); }

void kifmm_destroy(kifmm_handle h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->last_stream);
    if (h->events.made) {
        for (auto& row : h->events.ev)
            for (auto& e : row) (void)hipEventDestroy(e);
        for (auto& row : h->events.p2p)
            for (auto& e : row) (void)hipEventDestroy(e);
    }
    delete h;
}

const char* kifmm_status_string(int status) {
    static thread_local std::string msg;
    const char* base = "unknown status";
    switch (status) {
        case KIFMM_OK: base = "ok"; break;
        case KIFMM_ERR_ARG: base = "invalid argument"; break;
        case KIFMM_ERR_INPUT: base = "invalid input data"; break;
        case KIFMM_ERR_OOM: base = "out of device memory"; break;
        case KIFMM_ERR_HIP: base = "HIP runtime error"; break;
        case KIFMM_ERR_STATE: base = "invalid handle or state"; break;
    }
    msg = base;
    if (status != KIFMM_OK && !g_err.empty()) msg += ": " + g_err;
    return msg.c_str();
}

}  // extern "C"
