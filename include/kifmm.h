/*
 * kifmm.h -- C ABI of the MI355X KIFMM library (libkifmm.so).
 *
 * The library evaluates the long-range sum of the paper's eq. (1) with
 * sources equal to targets (Section 2.2): for N points x_i with scalar
 * charges q_i (the per-particle charge attribute of Section 2.4),
 *
 *     u_i = sum_{j : x_j != x_i} K(x_i - x_j) q_j,     E_i = -grad u (x_i),
 *
 * with K(r) = c/|r|; c = 1/(4 pi) for the Laplace/Coulomb kernel (the force
 * q_i E_i is eq. (3)) and c = -1 for gravity with G = 1 (m_i E_i is the
 * attractive force of eq. (4)).  The sum is approximated by the
 * kernel-independent fast multipole method of Section 2.2: an octree with at
 * most M points per leaf, an upward pass (P2M, M2M), a downward pass (M2L,
 * L2L, plus the adaptive-tree X list) and a leaf evaluation (L2P, the W list
 * and the near-field P2P), with densities on equivalent surfaces and
 * translation matrices computed from the kernel.
 *
 * Conventions for every entry point
 *  - All array pointers are DEVICE pointers (HIP global memory) unless the
 *    comment says "host".  Arrays are dense, row-major, in the caller's point
 *    order: positions [N][3] double, charges [N] float, field [N][3] float.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    kifmm_setup*, kifmm_rebuild and kifmm_set_clumps synchronise that
 *    stream (sizes and offsets are read back), as do the query and copy
 *    calls and kifmm_synchronize; the evaluation, adjoint and clump calls
 *    are asynchronous on it.  kifmm_evaluate and kifmm_backward
 *    run the near field on a second stream owned by the handle, forked from
 *    and joined back to `stream` with events, so their results are ordered
 *    on `stream` as if everything ran there.  One handle must not be used
 *    from two streams at once.
 *  - The caller owns every argument buffer; the library keeps no pointer to
 *    them after the call's work has run on the stream.  The handle owns its
 *    device copies of the positions, the tree, the lists, the operators and
 *    the work space, all freed by kifmm_destroy.
 *  - Outputs are overwritten, never accumulated into.
 *  - Every int-returning call returns KIFMM_OK (0) or a negative status; no
 *    C++ exception crosses the ABI.  After an error the handle (if one was
 *    returned) stays valid for kifmm_destroy.  kifmm_status_string gives a
 *    message for the last error of the calling thread.
 */
#ifndef KIFMM_H
#define KIFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kifmm_plan* kifmm_handle;

enum kifmm_kernel {
    KIFMM_LAPLACE = 0,   /* K = 1/(4 pi r): Coulomb, eq. (3) */
    KIFMM_GRAVITY = 1    /* K = -1/r, G = 1: gravity, eq. (4) */
};

enum kifmm_precision {
    KIFMM_FP32 = 0,        /* every far-field product in FP32 (MFMA f32) */
    KIFMM_SPLIT_BF16 = 1   /* M2L products as bf16 hi/lo splits (three bf16 MFMA
                              products, FP32 accumulation); all else FP32 */
};

enum kifmm_status {
    KIFMM_OK = 0,
    KIFMM_ERR_ARG = -1,     /* null required pointer, N < 1, p outside 2..8,
                               leaf_size < 1, max_depth outside 0..21, unknown
                               kernel or precision, bad root side */
    KIFMM_ERR_INPUT = -2,   /* non-finite position, point outside the explicit
                               root, non-monotone clump offsets */
    KIFMM_ERR_OOM = -3,     /* device allocation failed */
    KIFMM_ERR_HIP = -4,     /* a HIP runtime error (message kept) */
    KIFMM_ERR_STATE = -5    /* null handle or an unusable handle */
};

typedef struct {
    int adaptive;          /* 1 (default): a box is a leaf when it holds <= leaf_size
                              points or sits at max_depth.  0: every box at depth
                              min(max_depth, min{L : leaf_size 8^L >= N}) is a leaf. */
    int max_depth;         /* deepest level, 0..21 (default 21 = key resolution) */
    int precision;         /* enum kifmm_precision (default KIFMM_FP32) */
    double pinv_rtol;      /* singular values below pinv_rtol * sigma_1 are dropped
                              from the check-to-equivalent pseudoinverses (1e-7) */
    int explicit_root;     /* 0 (default): root cube from the bounding box; 1: use
                              root_lo/root_side */
    double root_lo[3];     /* root corner; must lie on the root_side/4096 grid */
    double root_side;      /* power of two; every point must satisfy
                              root_lo <= x <= root_lo + root_side */
    int profile;           /* 1: record per-phase HIP events on the stream
                              (kifmm_get_phase_times) */
    int periodic;          /* 1: the explicit root cube is the unit cell of a
                              system periodic in x, y and z (Section 2.4); Laplace
                              kernel only, explicit_root required, every point
                              inside the cell.  The potential is the lattice sum
                              read as the Ewald sum with conducting boundary (no
                              surface term); for a cell with net charge the
                              uniform neutralising background is implied.  Images
                              within one cell come from the lists (entries carry
                              the image shift, see kifmm_copy_list), images
                              further away from a root lattice operator, and the
                              non-harmonic part of the periodic kernel from the
                              sources' moments in closed form.  0 (default): free
                              space. */
    double m2l_rtol;       /* > 0: apply M2L in the truncated common basis of the 316
                              offset operators (left singular vectors of
                              [M2L(d_1) ... M2L(d_316)] with sigma >= m2l_rtol
                              sigma_1; the same basis on the source side since
                              M2L(-d) = M2L(d)^T, so kifmm_backward stays the exact
                              adjoint).  Used when its padded rank is a smaller M2L
                              tile than the surface (p = 6, 1e-6: 116 of 152 -> 128;
                              p = 8: 124 of 296 -> 128).  0 (default): the exact
                              operators. */
} kifmm_options;

/* Fill *opts with the defaults listed above. */
void kifmm_default_options(kifmm_options* opts);

/*
 * Build a plan: root cube, Morton keys, radix sort, octree (Section 2.2,
 * leaves with at most leaf_size = M points), interaction lists, and the
 * FP64 operator precompute (cached per kernel, p and pinv_rtol).
 *   positions  device, [N][3] double, caller order; rounded to FP32 for the
 *              floating-point work, used in FP64 for the integer keys.
 *   N          number of points (>= 1).
 *   kernel     enum kifmm_kernel.
 *   p          surface order 2..8: n = 6 (p-1)^2 + 2 samples per surface.
 *   leaf_size  M >= 1.
 *   opts       nullable (defaults).
 *   out        host; receives the handle (NULL on failure before allocation).
 * Synchronises `stream`.
 */
int kifmm_setup(const double* positions, int64_t N, int kernel, int p, int leaf_size,
                kifmm_handle* out);
int kifmm_setup_ex(const double* positions, int64_t N, int kernel, int p, int leaf_size,
                   const kifmm_options* opts, void* stream, kifmm_handle* out);

/*
 * Rebuild the tree and lists of an existing plan for new positions (same N,
 * kernel, p, leaf size and options); work space is reused where it fits.
 * This is the per-call re-tree of particles that move between long-range
 * evaluations (Section 2.4).  The sort starts from the previous build's
 * order: the keys are formed in that order, the points out of order with a
 * neighbour are sorted on their own and merged back into the rest (when the
 * rest is in order and they are at most a quarter of the points; otherwise
 * the full radix sort runs).  The result is the same order as a fresh
 * set-up's.  Synchronises `stream`.
 */
int kifmm_rebuild(kifmm_handle h, const double* positions, void* stream);

/* Select the M2L precision (enum kifmm_precision) for later calls. */
int kifmm_set_precision(kifmm_handle h, int precision);

/*
 * Forward evaluation (Section 2.2, all four steps after the tree):
 *   charges    device [N] float, caller order.
 *   potential  device [N] float or NULL.
 *   field      device [N][3] float (E = -grad u) or NULL.
 */
int kifmm_evaluate(kifmm_handle h, const float* charges, float* potential, float* field,
                   void* stream);

/*
 * Forward evaluation with dipole sources (the dipole granulates that eq. (1)
 * with other kernels covers): every point carries a charge q_j (or none) and
 * a dipole m_j, a dipole at y making psi(x) = -m . G(x - y), G = -grad K:
 *   u_i = sum_{j : x_j != x_i} [q_j K(x_i - x_j) - m_j . G(x_i - x_j)],  E = -grad u.
 *   charges    device [N] float or NULL (= 0), caller order.
 *   dipoles    device [N][3] float, caller order.
 *   potential, field as for kifmm_evaluate.
 * The same sweep as kifmm_evaluate, with the dipole parts in every point-to-
 * surface and point-to-point sum.  Afterwards kifmm_backward needs its
 * charges (the reused forward pass is gone).
 */
int kifmm_evaluate_dipoles(kifmm_handle h, const float* charges, const float* dipoles, float* potential,
                           float* field, void* stream);

/*
 * Forward evaluation with the field gradient, for the force on a dipole
 * (F = (m . grad) E for a curl-free field) and the other outputs of the
 * "other kernels" of eq. (1):
 *   charges     device [N] float or NULL, caller order.
 *   dipoles     device [N][3] float or NULL (at least one of the two given);
 *               a dipole m at y makes psi(x) = -m . G(x - y), as above.
 *   potential   device [N] float or NULL.
 *   field       device [N][3] float (E = -grad u) or NULL.
 *   field_grad  device [N][6] float or NULL: dE_a/dx_b = -d2u/dx_a dx_b,
 *               components (xx, yy, zz, xy, xz, yz).
 * The sweep of kifmm_evaluate (or of kifmm_evaluate_dipoles with dipoles);
 * the leaf evaluation also differentiates the equivalent densities and the
 * near field sums the pair Hessians.  Periodic plans add the moment term
 * (-4 pi c Q / (3 V) on the diagonal).  Afterwards kifmm_backward needs its
 * charges.
 */
int kifmm_evaluate_gradient(kifmm_handle h, const float* charges, const float* dipoles, float* potential,
                            float* field, float* field_grad, void* stream);

/*
 * Stokes flow of point forces (the tensor Stokeslet kernel that eq. (1)
 * covers, Section 2.2): for forces f_j at the plan's points in a fluid of
 * viscosity mu,
 *   u_i = 1/(8 pi mu) sum_{j : x_j != x_i} [ f_j / r + (r . f_j) r / r^3 ],  r = x_i - x_j.
 * The near lists are summed point to point with this kernel; the rest comes
 * from four charge evaluations of the plan's Laplace method (the harmonic
 * decomposition of the Stokeslet: with x' = x - o for any fixed o, the
 * charges f_x, f_y, f_z and x' . f give potentials psi_k and fields E(k),
 * and sum S f = (psi_a + x'_k E(k)_a - E(4)_a) / c).
 *   forces     device [N][3] float, caller order.
 *   viscosity  mu > 0.
 *   velocity   device [N][3] float, caller order.
 * Needs a free-space Laplace plan (KIFMM_ERR_STATE otherwise).  Two sweeps of
 * two right-hand sides each; afterwards kifmm_backward needs its charges.
 * The fourth charge is formed about each box's own centre c, (y - c) . f,
 * and every translation adds the shift of centres times the box's densities
 * of f_x, f_y, f_z; each target combines about its leaf centre, so no term
 * carries the distance to a far origin (with one origin the far terms grow
 * as |x - o| over the distance to the sources, about 12-fold at a million
 * clustered points).  Workspace beyond kifmm_evaluate: the first sweep's
 * densities of f_x, f_y and one float4 per point, kept by the plan.
 */
int kifmm_evaluate_stokes(kifmm_handle h, const float* forces, double viscosity, float* velocity, void* stream);

/*
 * The same Stokeslet sum together with the pressure of the flow,
 *   p_i = 1/(4 pi) sum_{j : x_j != x_i} (r . f_j) / r^3,  r = x_i - x_j,
 * which with the velocity satisfies mu lap u = grad p away from the forces.
 * Through the harmonic decomposition it is the trace of the fields of the
 * charges f_x, f_y, f_z, (E(1)_x + E(2)_y + E(3)_z) / (4 pi c), which the
 * velocity already computes; the near part is summed with the velocity's
 * pairs.
 *   pressure   device [N] float, caller order, or NULL (then exactly
 *              kifmm_evaluate_stokes).
 * Other arguments, requirements and errors as kifmm_evaluate_stokes.
 */
int kifmm_evaluate_stokes_ex(kifmm_handle h, const float* forces, double viscosity, float* velocity,
                             float* pressure, void* stream);

/*
 * Vector-Jacobian product of the discrete map (q, x) -> (u, E) of
 * kifmm_evaluate at the plan's positions with the tree frozen: given
 * grad_potential = dL/du and grad_field = dL/dE (either may be NULL = 0),
 * writes grad_charges = dL/dq [N] and grad_positions = dL/dx [N][3] (either
 * may be NULL).  Implemented as the transposed sweep: a sweep carries
 * monopole (dL/du) and dipole (dL/dE) sources beside the forward densities;
 * the plan's operators are symmetric, so the transposed sweep reuses them.
 *   charges  device [N] float, caller order: the forward densities are
 *            recomputed for these charges; or NULL: the charges and forward
 *            densities of the last kifmm_evaluate (or kifmm_backward with
 *            charges) on this handle are reused, which saves the forward
 *            sweep.  NULL after setup, kifmm_rebuild or kifmm_set_precision
 *            (before the next evaluation) is KIFMM_ERR_STATE.
 */
int kifmm_backward(kifmm_handle h, const float* charges, const float* grad_potential,
                   const float* grad_field, float* grad_charges, float* grad_positions,
                   void* stream);

/*
 * Clump aggregation (Section 2.4): pebble forces F_k = q_k E_k are summed
 * per clump, F_c = sum F_k and T_c = sum (x_k - X_c) x F_k, in FP64, over the
 * pebbles of each clump (a segmented reduction in a fixed order: a
 * deterministic result equal to the caller-order sum up to FP64 rounding).
 *   charges        device [N] float, field device [N][3] float (from
 *                  kifmm_evaluate), both caller order.
 *   clump_offsets  device [C+1] int64, CSR over caller order, offsets[0] = 0,
 *                  non-decreasing, offsets[C] <= N.  Checked on the device:
 *                  a clump whose row is not valid gets NaN force and torque,
 *                  and the next kifmm_synchronize returns KIFMM_ERR_INPUT.
 *   centers        device [C][3] double, the reference point X_c of each clump.
 *   force, torque  device [C][3] double.
 * The pebble positions are the plan's.  Asynchronous; the first call on a
 * plan allocates its partial-sum buffer (16 bytes per pebble or less).
 */
int kifmm_clump_reduce(kifmm_handle h, const float* charges, const float* field,
                       const int64_t* clump_offsets, int64_t C, const double* centers,
                       double* force, double* torque, void* stream);

/*
 * kifmm_clump_reduce for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it):
 * the same arguments, kernels and results, but the reduction's partial sums
 * live in a fixed device array of the library (4 MiB per device, held until
 * the process ends) instead of a buffer of the plan, and the call allocates
 * nothing.  Its limit is N <= 11,184,640 points (KIFMM_ERR_ARG beyond).  All
 * calls on one device share that array: calls that overlap on one device
 * (other streams, other handles) race and must be ordered by the caller.
 */
int kifmm_clump_reduce_noalloc(kifmm_handle h, const float* charges, const float* field,
                               const int64_t* clump_offsets, int64_t C, const double* centers,
                               double* force, double* torque, void* stream);

/*
 * Backward of kifmm_clump_reduce (the vector-Jacobian product of the Section
 * 2.4 aggregation) for given dL/dF_c and dL/dT_c, with r_k = x_k - X_c:
 *   grad_charges[k]   = dL/dF_c . E_k + dL/dT_c . (r_k x E_k)
 *   grad_field[k]     = q_k (dL/dF_c + dL/dT_c x r_k)
 *   grad_positions[k] = q_k (E_k x dL/dT_c)
 *   grad_centers[c]   = - sum_{k in c} grad_positions[k]
 * Arguments as for kifmm_clump_reduce (offsets checked the same way);
 * grad_force, grad_torque: device [C][3] double (either may be NULL = 0);
 * grad_charges [N] float, grad_field [N][3] float, grad_positions [N][3]
 * float, grad_centers [C][3] double (each may be NULL).  These are the direct
 * parts: the charge and position gradients of the whole map (q, x) ->
 * (F_c, T_c) add kifmm_backward with grad_field as its dL/dE.  Pebbles outside
 * every clump get zeros.  FP64 arithmetic; asynchronous.
 */
int kifmm_clump_backward(kifmm_handle h, const float* charges, const float* field,
                         const int64_t* clump_offsets, int64_t C, const double* centers,
                         const double* grad_force, const double* grad_torque, float* grad_charges,
                         float* grad_field, float* grad_positions, double* grad_centers, void* stream);

/*
 * Register the rigid clumps of Section 2.4 with the plan: clump c is the
 * caller-order points [clump_offsets[c], clump_offsets[c+1]) (device [C+1]
 * int64, offsets[0] = 0, non-decreasing, offsets[C] <= N; points after
 * offsets[C] belong to no clump).  The offsets are copied and checked here
 * (KIFMM_ERR_INPUT), so the clump calls below neither copy nor check them.
 * The membership stays with the plan through kifmm_rebuild; C = 0 removes it.
 * Synchronises `stream`.
 */
int kifmm_set_clumps(kifmm_handle h, const int64_t* clump_offsets, int64_t C, void* stream);

/*
 * Force and torque on every registered clump (Section 2.4): one evaluation of
 * the charges, then the FP64 aggregation of kifmm_clump_reduce.  The
 * evaluation leaves out the point-to-point pairs of two pebbles of one clump:
 * such a pair's forces are equal and opposite along the line joining the two
 * pebbles, so they add nothing to F_c or T_c, and leaving them out keeps
 * their (large, cancelling) rounding out of the sums.
 *   charges        device [N] float, caller order.
 *   centers        device [C][3] double (X_c).
 *   force, torque  device [C][3] double.
 *   field          device [N][3] float or NULL: receives the pebble fields
 *                  the sums used (the field at each pebble without the
 *                  point-to-point part of its own clump).
 * Asynchronous.  Keeps the forward state for kifmm_clump_forces_backward.
 */
int kifmm_clump_forces(kifmm_handle h, const float* charges, const double* centers, double* force,
                       double* torque, float* field, void* stream);

/*
 * Vector-Jacobian product of kifmm_clump_forces (tree frozen), for dL/dF_c and
 * dL/dT_c (device [C][3] double, either may be NULL = 0), at the charges of
 * the last kifmm_clump_forces on this handle (passed again: `charges`, the
 * same [N] float buffer contents):
 *   grad_charges [N] float, grad_positions [N][3] float, grad_centers [C][3]
 *   double (each may be NULL)
 * hold the whole gradient: the aggregation's direct parts plus the adjoint
 * sweep of its dL/dE (the same pairs left out).  KIFMM_ERR_STATE when the last
 * evaluation on the handle was not kifmm_clump_forces.  Asynchronous.
 */
int kifmm_clump_forces_backward(kifmm_handle h, const float* charges, const double* centers,
                                const double* grad_force, const double* grad_torque, float* grad_charges,
                                float* grad_positions, double* grad_centers, void* stream);

/*
 * Wait for the handle's work on `stream` and report input errors that
 * asynchronous calls found on the device since the last kifmm_synchronize
 * (invalid clump offsets: KIFMM_ERR_INPUT); clears them.
 */
int kifmm_synchronize(kifmm_handle h, void* stream);

/*
 * Sizes of the plan (host out[10]): boxes, leaves, depth, V-list pairs,
 * near-field point pairs (over the near lists, self pairs included), W-list pairs, X-list
 * pairs, U-list leaf pairs, N, surface points n.  The two pair counts are
 * taken on the first call after a build (two small kernels on the handle's
 * last stream, which the call then synchronises), not by the build itself.
 */
int kifmm_get_counts(kifmm_handle h, int64_t out[10]);

/*
 * Build statistics (host out[3]): out[0] tree builds of the plan (set-up and
 * rebuilds), out[1] builds that started from the previous build's order (a
 * rebuild with that order at hand), out[2] of those, the ones whose sort was
 * finished that way (the points out of order with a neighbour sorted on their
 * own and merged back into the rest); the others ran the full radix sort.
 * Either way the order is the same: by key, ties by caller index.
 */
int kifmm_get_build_stats(kifmm_handle h, int64_t out[3]);

/*
 * The M2L operators in use (host out[2]): out[0] = their rank (the number of
 * basis vectors kept with opts.m2l_rtol > 0, else the surface size n),
 * out[1] = the tile the M2L kernel runs at (the padded rank, or n padded).
 */
int kifmm_get_m2l_rank(kifmm_handle h, int64_t out[2]);

/*
 * The FP64 operators behind the plan (Section 2.2: the translation and
 * check-to-equivalent matrices computed from the kernel), for checks against
 * an independent computation.  Unit box, kernel 1/r; HOST buffers.
 *   which 0: singular values of K(uc, ue) (n values, descending); out[1] =
 *            the rank the pseudoinverses keep (sigma >= pinv_rtol sigma_1).
 *   which 1: singular values of [M2L(d_1) ... M2L(d_316)] (n values,
 *            descending, from the eigenvalues of the sum of M2L(d) M2L(d)^T);
 *            out[1] = the rank kept with opts.m2l_rtol (KIFMM_ERR_STATE when
 *            the plan has m2l_rtol = 0).
 *   which 2: the pseudoinverse UC2E of K(uc, ue), n x n row-major.
 *   values   host, cap doubles, or NULL to ask for the size; out[0] = the
 *            number of values (KIFMM_ERR_ARG when cap is smaller).
 */
int kifmm_get_operator(kifmm_handle h, int which, double* values, int64_t cap, int64_t out[2]);

/*
 * Copy the tree to HOST buffers (each may be NULL), sized by kifmm_get_counts:
 *   keys [N] uint64 sorted Morton keys, perm [N] int64 (sorted position ->
 *   caller index), level/anchor/begin/end/parent/is_leaf per box (anchor is
 *   [B][3]; boxes are numbered level by level in Morton order), root[4] =
 *   (lo_x, lo_y, lo_z, side).  Synchronises the handle's last stream.
 */
int kifmm_copy_tree(kifmm_handle h, uint64_t* keys, int64_t* perm, int32_t* level,
                    int32_t* anchor, int64_t* begin, int64_t* end, int64_t* parent,
                    int8_t* is_leaf, double* root);

/*
 * Copy one interaction list (which = 'U', 'V', 'W' or 'X', or 'N' for the
 * near list that the point-to-point pass walks) as host CSR over boxes:
 * offsets [B+1] int64, indices [pairs] int64 (source boxes, ascending within a
 * row of U, V, W, X; a near row is U, then X, then W entries).  A W/X pair
 * (box A, finer box F: F in W(A), A in X(F)) is summed point to point in both
 * directions, and so sits in the near lists of the leaves F and A, when F is
 * a leaf holding at most n points (n the surface size); the other W/X pairs
 * go through the expansions.  Pass offsets only (indices NULL) to size the
 * second call.
 * Periodic plans: an entry names box (entry & (2^26 - 1)) shifted by s root
 * widths, s in {-1,0,1}^3 coded in entry >> 26 as (9 (sx+1) + 3 (sy+1) +
 * (sz+1) + 14) mod 27 (0 = unshifted, so free-space entries are plain box
 * indices); rows ascend in the coded value.
 */
int kifmm_copy_list(kifmm_handle h, char which, int64_t* offsets, int64_t* indices);

/*
 * Per-phase device times in ms of the last evaluate/backward (host out[n]):
 * 0 P2M, 1 upward M2M+UC2E (and, with opts.m2l_rtol, the projection onto
 * the M2L basis), 2 P2L, 3 M2L, 4 L2L+DC2E (and the expansion out of the M2L
 * basis), 5 L2P+M2P (with the
 * final combination), 6 P2P (on the near-field stream, concurrent with 0-4),
 * 7 whole call.  Needs opts.profile = 1; returns the number written (0 when
 * the call recorded nothing).  Waits for that call's events.
 */
int kifmm_get_phase_times(kifmm_handle h, float* out, int n);

/*
 * The same for the profiled call `back` calls before the last (0 = the last,
 * up to 63: the plan keeps the events of its last 64 profiled evaluation,
 * adjoint and clump-force calls), so that a run of calls can be timed
 * without waiting between them.  KIFMM_ERR_ARG when that call is not kept.
 */
int kifmm_get_phase_times_at(kifmm_handle h, int back, float* out, int n);

/* Release the handle and everything it owns (NULL is accepted). */
void kifmm_destroy(kifmm_handle h);

/* Message for a status code (with detail for the calling thread's last error). */
const char* kifmm_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* KIFMM_H */
