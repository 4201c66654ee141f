// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <string>
#include <functional>
#include <vector>

#include "../../include/kifmm.h"

namespace kifmm {

constexpr int kBits = 21;              // key bits per axis
constexpr int kNumV = 316;             // far offsets in [-3,3]^3 minus [-1,1]^3
constexpr int kVPerOct = 189;          // V-list offsets reachable from one octant
constexpr int kMaxLevels = 22;
constexpr int kM2LSplit = 4;          // M2L V slots split over this many blocks per tile
constexpr int kM2LSplitMax = 16;      // ... and up to this many for small trees
constexpr int kM2LFill = 2048;        // M2L blocks wanted before the split stops growing
constexpr int kMomentBlocks = 256;    // blocks of the periodic moment reduction
// fixed device scratch of kifmm_clump_reduce_noalloc (per device, for the
// process lifetime): the clump reduction's segment partials, 96 bytes per
// block of 256 pebbles, so at most 11,184,640 pebbles
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
constexpr int kMaxDevices = 64;

// Error carrying a status code; caught at the ABI.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define KIFMM_HIP(call)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::kifmm::Error(e_ == hipErrorOutOfMemory ? KIFMM_ERR_OOM : KIFMM_ERR_HIP, \
                                 std::string(#call) + ": " + hipGetErrorString(e_));      \
    } while (0)

// List entries with periodic images: entry = box | code << kShiftBits, the
// image shift s in {-1,0,1}^3 (in root widths) coded as
// (9 (sx+1) + 3 (sy+1) + (sz+1) + 14) mod 27, so that the unshifted image has
// code 0 and free-space entries are plain box indices.
constexpr int kShiftBits = 26;
constexpr int kBoxMask = (1 << kShiftBits) - 1;

__host__ __device__ inline int img_encode(int box, int sx, int sy, int sz) {
    const int raw = 9 * (sx + 1) + 3 * (sy + 1) + (sz + 1);
    return box | (((raw + 14) % 27) << kShiftBits);
}
__host__ __device__ inline int img_box(int e) { return e & kBoxMask; }
__host__ __device__ inline void img_shift(int e, int& sx, int& sy, int& sz) {
    const int raw = ((e >> kShiftBits) + 13) % 27;
    sx = raw / 9 - 1;
    sy = (raw / 3) % 3 - 1;
    sz = raw % 3 - 1;
}
// the same box seen from the other side: shift negated
__host__ __device__ inline int img_flip(int e) {
    int sx, sy, sz;
    img_shift(e, sx, sy, sz);
    return img_encode(img_box(e), -sx, -sy, -sz);
}

// Grow-only device buffer.
// A few pinned host words for the small device-to-host reads of the tree
// build (allocated once per plan with hipHostMalloc, freed with the plan).
struct HostWords {
    void* p = nullptr;
    HostWords() = default;
    HostWords(const HostWords&) = delete;
    HostWords& operator=(const HostWords&) = delete;
    ~HostWords() {
        if (p) (void)hipHostFree(p);
    }
    unsigned long long* get() {
        if (!p) KIFMM_HIP(hipHostMalloc(&p, 512, hipHostMallocDefault));
        return static_cast<unsigned long long*>(p);
    }
};

struct DBuf {
    void* p = nullptr;
    size_t cap = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    // Make room for `bytes` (contents are not preserved).
    void* ensure(size_t bytes) {
        if (bytes == 0) bytes = 256;
        if (bytes > cap) {
            release();
            size_t b = (bytes + 255) & ~size_t(255);
            KIFMM_HIP(hipMalloc(&p, b));
            cap = b;
        }
        return p;
    }
    // Grow keeping the first `keep` bytes.
    void* grow(size_t bytes, size_t keep, hipStream_t s) {
        if (bytes <= cap) return p;
        size_t b = ((bytes + bytes / 2) + 255) & ~size_t(255);
        void* q = nullptr;
        KIFMM_HIP(hipMalloc(&q, b));
        if (p && keep) KIFMM_HIP(hipMemcpyAsync(q, p, keep, hipMemcpyDeviceToDevice, s));
        if (p) {
            KIFMM_HIP(hipStreamSynchronize(s));
            (void)hipFree(p);
        }
        p = q;
        cap = b;
        return p;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Operators of one (p, pinv_rtol): built on the host in FP64, stored in FP32
// (and bf16 hi/lo for M2L) on the device.  Unit-box coordinates, kernel 1/r.
struct Operators {
    int p = 0, n = 0, npad = 0, rank = 0;
    double tau = 0;
    DBuf surf;         // float4 [2][npad]: rho=1.05 surface, rho=2.95 surface (w = 0)
    // check-to-equivalent factors in chain order ([ob][rb][64] x 16 B):
    DBuf uc2e_w1;      // Sigma^-1 U^T          (UC2E = V W1)
    DBuf uc2e_v;       // V
    DBuf dc2e_w1;      // Sigma^-1 V^T          (DC2E = UC2E^T = U W1d)
    DBuf dc2e_v;       // U
    // translations in gather-fragment order ([op][kc][rb][2][64] x 16 B):
    DBuf m2m;          // 8 octants: parent uc <- child ue
    DBuf l2l;          // 8 octants: child dc <- parent de (includes the factor 1/2 of the child width)
    DBuf m2l_f32;      // [316][npad/32 chunks][npad/16 row blocks][2][64] x 16 B (FP32 fragments)
    DBuf m2l_bf16;     // same shape, bf16 hi half then lo half
    std::vector<double> sigma;   // singular values of K(uc, ue), descending
    std::vector<double> svd_u, svd_v;   // its singular vectors (n x n row-major, FP64)
};

// M2L in a truncated common basis Q (n x k, the left singular vectors of
// [M2L(d_1) ... M2L(d_316)] with sigma >= rtol * sigma_1; since M2L(-d) =
// M2L(d)^T the same basis serves the source side): the sweep projects the
// upward densities, phi_k = Q^T phi_u, applies the k x k cores Q^T M2L(d) Q
// and expands the result, psi += Q psi_k.  kp is the padded rank, one of the
// tile sizes the M2L kernel is built for; kp = 0 means the basis does not pay.
struct M2LBasis {
    int k = 0, kp = 0;
    std::vector<double> sigma;   // singular values of [M2L(d_1) ... M2L(d_316)] (unit operators), descending
    DBuf q;           // float [NP][kp]: Q row-major, zero-padded (operand of the expansion psi += Q psi_k)
    DBuf qt;          // float [kp][NP]: Q^T row-major, zero-padded (operand of the projection phi_k = Q^T phi)
    DBuf core_f32;    // [316] cores in gather-fragment order at kp (FP32)
    DBuf core_bf16;   // the same, bf16 hi/lo
};
const M2LBasis& get_m2l_basis(int p, double tau, double rtol);

// Periodic root operator (unit cell, FP64 [n][n] row-major on the device):
// the root downward equivalent density from the root upward density for
// every image at cube distance two or more, DC2E F(dc - ue).
const DBuf& get_lattice_operator(int p, double tau);

// Returns the (cached, process-wide) operators for this device.
const Operators& get_operators(int p, double tau);

// Host FP64 one-sided Jacobi SVD of a square row-major matrix A (n x n):
// A = U diag(S) V^T, S descending.  U, V row-major n x n.
void jacobi_svd(int n, const double* A, double* U, double* S, double* V);

// Surfaces in unit-box coordinates: boundary points of the p^3 grid,
// i slowest, k fastest, scaled by rho about the centre.
std::vector<double> unit_surface(int p, double rho);

struct LevelInfo {
    int64_t start = 0, count = 0;     // boxes of this level: [start, start+count)
    int64_t nl_start = 0, nl_count = 0;  // non-leaf boxes of this level in nonleaf[]
};

// Phase events of the last kRing profiled calls (a ring, so that a caller
// can read them after a run of calls without synchronising in between): per
// call ev[0] start, ev[1..5] after P2M, upward, P2L, M2L, downward on the
// caller's stream, ev[6] after it has joined the near-field stream, ev[7]
// after the leaf evaluation; p2p[0..1] around the near field on the side stream.
struct PhaseEvents {
    static constexpr int kRing = 64;
    hipEvent_t ev[kRing][8] = {};
    hipEvent_t p2p[kRing][2] = {};
    bool valid[kRing] = {};   // the slot holds a finished call's events
    int cur = kRing - 1;      // slot of the last (or running) call
    int64_t calls = 0;
    bool made = false;
};

// The second stream the near field runs on, forked from and joined to the
// caller's stream with events (default priority).
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    SideStream() = default;
    SideStream(const SideStream&) = delete;
    SideStream& operator=(const SideStream&) = delete;
    ~SideStream() {
        if (s) (void)hipStreamSynchronize(s);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (s) (void)hipStreamDestroy(s);
    }
    void make() {
        if (s) return;
        KIFMM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        KIFMM_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        KIFMM_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    }
};

}  // namespace kifmm

// The plan behind a kifmm_handle.
struct kifmm_plan {
    int kernel = 0;
    double c = 0;
    int p = 0, n = 0, npad = 0, leaf = 0;
    kifmm_options opt{};
    int64_t N = 0;
    double lo[3] = {0, 0, 0}, side = 1;
    int depth = 0;
    int64_t B = 0, nleaves = 0;
    bool periodic = false;  // the root cube is the unit cell of a periodic system
    int64_t bfar = 0;       // first box with a downward density (level 2, or the root when periodic)
    std::vector<kifmm::LevelInfo> lev;
    int64_t counts[10] = {};
    bool pairs_counted = false;   // counts[3] and counts[4] (V pairs, P2P pairs) are taken on request
    hipStream_t last_stream = nullptr;
    const kifmm::Operators* ops = nullptr;
    const kifmm::M2LBasis* cm = nullptr;   // compressed M2L in use (null: the exact operators)
    kifmm::HostWords host;   // pinned words for small read-backs

    // points
    kifmm::DBuf x64;        // double [N][3] caller order (copy)
    kifmm::DBuf xs;         // float4 [N] sorted (x, y, z, 0)
    kifmm::DBuf perm;       // int32 [N] sorted -> caller
    kifmm::DBuf keys;       // uint64 [N] sorted
    // boxes
    kifmm::DBuf bx_anchor;  // int4 [B] (ax, ay, az, level)
    kifmm::DBuf bx_range;   // int2 [B] (begin, end)
    kifmm::DBuf bx_parent;  // int32 [B]
    kifmm::DBuf bx_child;   // int2 [B] (first child, child mask)
    kifmm::DBuf bx_leaf;    // int32 [B] 0/1
    kifmm::DBuf bx_mkey;    // uint64 [B] Morton key of the anchor at the box's level
    kifmm::DBuf nonleaf;    // int32 [.] non-leaf boxes, level by level
    kifmm::DBuf leaves;     // int32 [nleaves] leaf boxes
    // lists
    kifmm::DBuf coll;       // int32 [B][27]
    kifmm::DBuf cal;        // int32 [B][26] coarse adjacent leaves (-1 padded)
    kifmm::DBuf vdense;     // int32 [B - start(2)][189] V sources by octant-local offset slot
    kifmm::DBuf u_off, u_idx, w_off, w_idx, x_off, x_idx;   // CSR over boxes, int32
    kifmm::DBuf readback;   // staging words of the tree build's read-backs
    kifmm::DBuf xflag;   // [B + 1] int32: 1 for the boxes the P2L kernel writes (X lists not summed directly)
    kifmm::DBuf n_off, n_idx;   // near lists: U plus the W/X pairs summed point to point
    kifmm::DBuf wf_off, wf_idx; // W lists of the leaf evaluation (the other W pairs)
    kifmm::DBuf xboxes;     // int32 boxes with a non-empty X list
    kifmm::DBuf items_near, items_far;   // int2 (leaf, first target) work items, heaviest first
    kifmm::DBuf item_tmp;
    int64_t n_items = 0;
    int64_t n_xboxes = 0;
    // densities: [rhs][B][npad]
    kifmm::DBuf psi_u, phi_u, psi_d, phi_d;
    kifmm::DBuf phi_k;      // compressed M2L: projected upward densities [rhs][B][kp]
    kifmm::DBuf psi_m;      // M2L partial check potentials [split][rhs][B][npad]
    int m2l_split_used = kifmm::kM2LSplit;
    int m2l_split_cap = kifmm::kM2LSplit;   // partial buffers allocated
    // per-evaluation work
    kifmm::DBuf pts;        // float4 [N] sorted (x, y, z, q)
    kifmm::DBuf src2;       // float4 [N] sorted (ubar, Ebar) for the adjoint sweep
    kifmm::DBuf nearv;      // float4 [N] sorted near-field part: (u, E) or (xbar, qbar)
    kifmm::DBuf nearg;      // float [N][6] sorted near-field part of dE/dx (gradient calls only)
    kifmm::DBuf mom;        // periodic: double [rhs][16] source moments about the cell centre
    kifmm::DBuf mom_part;   // their per-block partial sums
    // scratch
    kifmm::DBuf tmp_a, tmp_b, tmp_c, tmp_d, tmp_e, tmp_f, scan_tmp, flag, pair_cnt;
    kifmm::DBuf resort;     // re-sort from the previous order: flags, offsets, the two subsequences
    bool sorted_valid = false;   // perm holds the order of the last build (same N)
    int64_t builds = 0, resort_steps = 0, resort_hits = 0;   // builds; those that tried / completed the re-sort
    kifmm::PhaseEvents events;
    kifmm::SideStream nearq;   // near-field stream
    bool fwd_valid = false;   // densities of right-hand side 0 and pts hold the last forward pass
    bool fwd_excl = false;    // ... and that pass left out the pairs of pebbles of one clump
    // input errors found on the device (clump offsets): int word, cleared by kifmm_synchronize
    kifmm::DBuf status;
    // registered clumps (kifmm_set_clumps)
    int64_t clumps = 0;
    kifmm::DBuf clump_off;    // int64 [C+1] CSR over caller order
    kifmm::DBuf cid;          // int32 [N] clump of each caller-order point (-1: none)
    kifmm::DBuf cid_s;        // int32 [N] sorted clump keys (unique negative values outside clumps)
    kifmm::DBuf clump_part;   // segment partials of the clump reductions [blocks][2][6] double
    kifmm::DBuf clump_E;      // float [N][3] pebble fields of the last kifmm_clump_forces
    kifmm::DBuf clump_Eb;     // float [N][3] its adjoint field sources
    // Stokeslet evaluation
    kifmm::DBuf stk;          // float4 [N] sorted forces
    kifmm::DBuf stk_near;     // float4 [N] sorted near-field velocity
    kifmm::DBuf stk_far;      // float [4][N] potentials, [4][N][3] fields of the harmonic charges (sorted order)
    kifmm::DBuf stk_keep;     // float: the first sweep's upward, compressed and downward densities of f_x, f_y
    kifmm::DBuf stk_frame;    // float4 [N] sorted x - (centre of the point's leaf)
};

namespace kifmm {

// ---- tree.hip
void build_tree(kifmm_plan* P, const double* positions, hipStream_t s);
// V-list pairs and near-field point pairs of the current lists into
// counts[3], counts[4] (synchronises s)
void count_pairs(kifmm_plan* P, hipStream_t s);
// offset (in box widths) from a box at octant o to the source of its V slot j
void v_slot_offset(int o, int j, int d[3]);
// ---- farfield.hip
// Per-box frames of the Stokeslet's fourth harmonic charge (x - c).f, the
// right-hand side 1 of the second Stokes sweep: its sources are formed about
// each box's own centre c, and each translation from box A to box B adds
// (c_A - c_B) times A's densities of the three force components, so that no
// value carries the distance to a distant origin.
struct StokesFrames {
    const float4* frc = nullptr;   // sorted forces (x, y, z, -)
    const float* up[3] = {};       // upward equivalent densities of f_x, f_y, f_z, [B][NP]
    const float* kp[3] = {};       // their compressed M2L sources, [B][KP] (compressed M2L only)
    const float* dn[3] = {};       // downward equivalent densities, [B][NP]
};
void run_sweep(kifmm_plan* P, int r0, int r1, hipStream_t s, bool record, const std::function<void()>& between,
               const StokesFrames* sf = nullptr);
// leaf evaluation; adds the near-field part and writes the caller-order
// outputs (forward: potential, field; backward: grad_charges, grad_positions)
// (near = false: the near-field part is not added)
// (sf: the W-list sources of right-hand side rhs are shifted into the
// target leaf's frame as for the Stokes sweep)
// (sorted: the outputs are written in sorted point order, not caller order)
void run_far_eval(kifmm_plan* P, bool backward, float* out_a, float* out_b, hipStream_t s, int rhs = 0,
                  bool accumulate = false, bool near = true, const StokesFrames* sf = nullptr,
                  bool sorted = false);
// leaf evaluation with the field gradient (densities of right-hand side rhs)
void run_far_grad(kifmm_plan* P, float* pot, float* field, float* grad, hipStream_t s, int rhs);
// ---- nearfield.hip
// sorted points (x, y, z, q) when `charges` is given or `points` is set (q = 0
// for null charges), and for `adjoint` the sorted (gpot, gfield) sources
void launch_gather(kifmm_plan* P, const float* charges, const float* gpot, const float* gfield,
                   bool adjoint, hipStream_t s, bool points = false);
// excl: pairs of points with equal sorted clump keys (cid_s) are left out
void launch_p2p_forward(kifmm_plan* P, hipStream_t s, bool excl = false);
void launch_p2p_backward(kifmm_plan* P, hipStream_t s, bool excl = false);
void launch_p2p_dipoles(kifmm_plan* P, hipStream_t s);
// Stokeslet sources (pass 0: f_x, f_y and the sorted forces; pass 1: f_z) and the Stokeslet near field
void launch_gather_stokes(kifmm_plan* P, const float* forces, int pass, hipStream_t s);
void launch_p2p_stokes(kifmm_plan* P, double viscosity, hipStream_t s);
// x - (centre of its leaf) of every sorted point, into stk_frame
void launch_stokes_frames(kifmm_plan* P, hipStream_t s);
// velocity from the harmonic potentials and fields (caller order, the fourth
// about each point's leaf centre) and the near part
void launch_stokes_combine(kifmm_plan* P, double viscosity, float* velocity, float* pressure, hipStream_t s);
// u, E and dE/dx of monopoles (pts.w, or src2.x with `dipoles`) and dipoles (src2.yzw)
void launch_p2p_gradient(kifmm_plan* P, bool dipoles, hipStream_t s);
// ---- clump.hip
// Per-clump sums over the CSR offsets `off` (caller order); with `cid` (the
// registered caller-order clump ids) the offsets are trusted, without it
// they are checked on the device (errors into P->status).  `part` holds
// clump_scratch_bytes(N, 6) bytes.
void launch_clump_reduce(kifmm_plan* P, const float* q, const float* E, const int64_t* off, const int* cid, int64_t C,
                         const double* centers, double* F, double* T, double* part, hipStream_t s);
// `acc`: grad_charges and grad_positions are added to, not overwritten
void launch_clump_backward(kifmm_plan* P, const float* q, const float* E, const int64_t* off, const int* cid,
                           int64_t C, const double* centers, const double* Fb, const double* Tb, float* qb,
                           float* Eb, float* xb, bool acc, double* Xb, double* part, hipStream_t s);
size_t clump_scratch_bytes(int64_t N, int nv);
// device address of the fixed scratch on the current device (looked up once per device)
void* noalloc_scratch();
// caller-order clump ids from checked device offsets
void set_clump_ids(kifmm_plan* P, const int64_t* off_dev, int64_t C, hipStream_t s);
// sorted clump keys for the current tree (after a build)
void launch_clump_ids(kifmm_plan* P, hipStream_t s);
// ---- api.cpp
void record_phase(kifmm_plan* P, int idx, hipStream_t s);

}  // namespace kifmm
