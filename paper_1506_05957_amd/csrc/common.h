// Internal declarations shared by the fmmbem HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fmmbem.h"
#include "harmonics.h"

namespace fmmbem {

// Block of the Arnoldi reductions (and of every kernel that sums their
// partials again): 256 threads.
constexpr int DOT_BLOCK = 256;
constexpr int DOT_NWV = DOT_BLOCK / 64;

// out[j] = sum_b part[j nb + b] for j < nv, into LDS, in a block of DOT_BLOCK
// threads (all of them take part): the waves take the vectors four at a time,
// lanes stride over b, then a shuffle tree.  The order is fixed, so every
// block that sums the same partials gets the same bits.
__device__ inline void block_sums(const double *__restrict__ part, int nb, int nv, double *__restrict__ out)
{
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int jb = 0; jb < nv; jb += 4 * DOT_NWV) {
        double t[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = lane; k < nb; k += 64) {
            double v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = jb + r * DOT_NWV + wv;
                v[r] = j < nv ? part[(int64_t)j * nb + k] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                t[r] += v[r];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                t[r] += __shfl_down(t[r], off, 64);
        if (lane == 0)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = jb + r * DOT_NWV + wv;
                if (j < nv)
                    out[j] = t[r];
            }
    }
}

// An Arnoldi normalisation folded into the charges of the next mat-vec: the
// input is w / |w|, |w|^2 = sum of the nb partials partn (the last Arnoldi
// step's), stored to nrm2_out; all null: no normalisation.
struct NormIn {
    const double *w = nullptr;
    const double *partn = nullptr;
    int nb = 0;
    double *nrm2_out = nullptr;
};

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define FB_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            throw ::fmmbem::Error(FMMBEM_EDEVICE, std::string(#call) + ": " +                 \
                                                      hipGetErrorString(e_));                 \
    } while (0)

#define FB_REQUIRE(cond, code, msg)                                                           \
    do {                                                                                      \
        if (!(cond))                                                                          \
            throw ::fmmbem::Error((code), (msg));                                             \
    } while (0)

// Number of m >= 0 coefficients of an expansion of order p.
__host__ __device__ constexpr inline int ncoef(int p) { return (p + 1) * (p + 2) / 2; }
__host__ __device__ constexpr inline int cidx(int n, int m) { return n * (n + 1) / 2 + m; }

constexpr int P_MAX = FMMBEM_P_MAX;
constexpr int P_MAX_FP32 = FMMBEM_P_MAX_FP32;
constexpr int NC_MAX = ncoef(P_MAX);
// longest chain of boxes (leaf and its ancestors down from the coarsest M2L
// target level) that the fused downward pass of one leaf takes, and the
// int32 fields of its per-leaf record: first target, end target, level,
// chain length, the chain (leaf first), the chain's octants (3 bits each), pad
constexpr int DOWN_LEAF_MAXC = 8;
constexpr int LEAF_REC = 16;
static_assert(4 + DOWN_LEAF_MAXC + 1 <= LEAF_REC, "leaf record");
// sources per P2P chunk (one LDS tile of a wave)
constexpr int P2P_TILE = 128;

// Where device memory comes from: the caller's callbacks (fmmbem_params
// alloc/free/alloc_user) or, when alloc is null, hipMalloc/hipFree.
struct DevAlloc {
    void *(*alloc)(size_t, void *) = nullptr;
    void (*free)(void *, void *) = nullptr;
    void *user = nullptr;
    void *get(size_t b) const
    {
        void *p = nullptr;
        if (alloc) {
            p = alloc(b, user);
            if (!p)
                throw Error(FMMBEM_ENOMEM, "caller allocator returned NULL for " + std::to_string(b) + " bytes");
            if (reinterpret_cast<uintptr_t>(p) % 256 != 0) {
                free(p, user);
                throw Error(FMMBEM_EINVAL, "caller allocator returned memory not aligned to 256 bytes");
            }
            return p;
        }
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess)
            throw Error(FMMBEM_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed: " +
                                           hipGetErrorString(e));
        return p;
    }
    void put(void *p) const
    {
        if (!p)
            return;
        if (alloc)
            free(p, user);
        else
            (void)hipFree(p);
    }
};

// Pinned, device-mapped host memory (the Hessenberg columns): hipHostMalloc,
// or the provider installed for the calling thread when there is one (the
// request loop keeps its own, because hipHostFree waits for the whole device
// while other requests run).  The provider is recorded with the buffer, so it
// goes back the same way from any thread.
struct PinnedProvider {
    void *(*get)(size_t bytes, void *user);
    void (*put)(void *p, void *user);
    void *user;
};
extern thread_local const PinnedProvider *t_pinned;
inline double *pinned_get(size_t bytes, const PinnedProvider **src)
{
    *src = t_pinned;
    void *p = nullptr;
    if (t_pinned) {
        p = t_pinned->get(bytes, t_pinned->user);
        if (!p)
            throw Error(FMMBEM_ENOMEM, "pinned host allocation failed");
    } else {
        hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocMapped);
        if (e != hipSuccess)
            throw Error(FMMBEM_ENOMEM, std::string("hipHostMalloc failed: ") + hipGetErrorString(e));
    }
    return static_cast<double *>(p);
}
inline void pinned_put(void *p, const PinnedProvider *src)
{
    if (!p)
        return;
    if (src)
        src->put(p, src->user);
    else
        (void)hipHostFree(p);
}

// Device buffers owned by a context; freed in reverse order on destruction.
struct DevArena {
    DevAlloc al;
    std::vector<void *> ptrs;
    int64_t bytes = 0;
    DevArena() = default;
    explicit DevArena(const DevAlloc &a) : al(a) {}
    DevArena(const DevArena &) = delete;
    DevArena &operator=(const DevArena &) = delete;
    template <typename T> T *alloc(size_t n) {
        size_t b = n * sizeof(T);
        if (b == 0)
            b = 16;
        ptrs.reserve(ptrs.size() + 1);  // a throw after the allocation would leak it
        void *p = al.get(b);
        ptrs.push_back(p);
        bytes += (int64_t)b;
        return static_cast<T *>(p);
    }
    void release() {
        for (auto it = ptrs.rbegin(); it != ptrs.rend(); ++it)
            al.put(*it);
        ptrs.clear();
        bytes = 0;
    }
};

// The octree and lists in sorted (Morton) order, as built on the device.
// first unit of each of the 8 XCD groups of a launch, and the end
struct XcdGroups {
    int32_t b[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    int32_t max_count() const
    {
        int32_t m = 0;
        for (int x = 0; x < 8; ++x)
            m = b[x + 1] - b[x] > m ? b[x + 1] - b[x] : m;
        return m;
    }
};

struct Tree {
    int64_t nt = 0;
    int32_t nbox = 0, nlevels = 0, nleaf = 0, max_leaf = 0;
    std::vector<int32_t> level_begin;  // boxes of level l are [level_begin[l], level_begin[l+1])
    double cube[4] = {0, 0, 0, 1};     // lower corner, side
    // device
    int32_t *perm = nullptr;      // [nt] sorted -> caller
    uint64_t *keys = nullptr;     // [nt]
    int32_t *box_i = nullptr;     // [nbox][6] level, begin, end, parent, child0, nchild
    double *box_r = nullptr;      // [nbox][5] cx, cy, cz, R, G
    int32_t *leaves = nullptr;    // [nleaf] box ids of leaves, box order
    int32_t *panel_leaf = nullptr;// [nt] leaf of each sorted panel
    int64_t n_m2l = 0, n_p2p = 0;
    int32_t *m2l_ptr = nullptr, *m2l_src = nullptr;  // CSR over all boxes
    int32_t *p2p_ptr = nullptr, *p2p_src = nullptr;  // CSR over all boxes (non-leaves empty)
    int32_t *m2l_pairs = nullptr, *p2p_pairs = nullptr;  // [n][2] sorted (target, source)
    // P2P work units: up to 64 targets of one leaf, with the leaf's P2P
    // sources as chunks of at most P2P_TILE consecutive sources of one source
    // leaf, in decreasing size order
    int32_t n_unit = 0;
    int64_t n_chunk = 0;
    int4 *p2p_unit = nullptr;     // [n_unit] first target, end target, first chunk, end chunk
    // launch order of the on-the-fly P2P: block b runs unit p2p_xcd.b[b % 8] +
    // b / 8 of XCD group b % 8 (groups of consecutive units with equal work,
    // heaviest unit first within a group).  A unit whose work exceeds the cap
    // is cut into pieces (chunk ranges of the same targets) that write partial
    // sums to slots of p2p_part, added in piece order by k_p2p_pieces
    XcdGroups p2p_xcd;
    int32_t *p2p_dst = nullptr;   // [n_unit] -1: the unit writes y_near; else its partial slot
    int32_t n_slot = 0, n_split = 0;
    double *p2p_part = nullptr;   // [n_slot][3][64] partial sums of the pieces
    int4 *p2p_split = nullptr;    // [n_split] first target, target count, first slot, pieces
    int2 *p2p_chunk = nullptr;    // [n_chunk] first source, count | 1 << 16 if it is the target's own leaf
    float4 *p2p_choff = nullptr;  // [n_chunk] target leaf centre - source leaf centre (FP32), 0
    // host copies of small metadata
    std::vector<int32_t> h_box_i;
    std::vector<double> h_box_r;
    std::vector<int32_t> h_leaves;
    int64_t p2p_interactions = 0;
};

struct Geometry {
    // sorted order, device
    double *tc = nullptr;    // [3][nt] centroids (SoA)
    double *S = nullptr;     // [nt] areas
    double *vtx = nullptr;   // [nt][9] panel vertices v0, v1, v2
    double *sp = nullptr;    // [4][nsrc] Gauss points x, y, z and weights q_k S_j
    double *nrm = nullptr;   // [3][nt] outward unit normals (v1 - v0) x (v2 - v0) / |.|
    float *tc32 = nullptr;   // [3][nt] centroid - leaf centre (FP32)
    float *sp32 = nullptr;   // [4][nsrc] Gauss point - leaf centre, weight (FP32)
};

struct Correction {
    int64_t nnz = 0;
    int32_t *ptr = nullptr;  // [nt + 1] by sorted target
    int32_t *col = nullptr;  // [nnz] sorted source panel
    int32_t *col_orig = nullptr;  // [nnz] the same panel in the caller's order
    double *val = nullptr;   // [nnz] (Laplace) or [nnz][9] (Stokes), without the kernel prefactor
    float *val32 = nullptr;  // the same values rounded to FP32, read by the FP32 mat-vecs
};

struct Timing {
    uint32_t mask = 0;  // bit s: stage s is timed
    double t_ms[FMMBEM_N_STAGES] = {0};
    int64_t launches[FMMBEM_N_STAGES] = {0};
    double flops[FMMBEM_N_STAGES] = {0};
    // pending event pairs, resolved at the next get or when the pool fills
    struct Pending { hipEvent_t a, b; int stage; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
};

// M2L pairs grouped by translation (translations.hip)
constexpr int M2L_CHUNK = 64;
struct M2LPlan {
    int q = 0;                          // tables hold I_n^m for n <= q = 2 p_max
    int n_trans = 0, n_chunks = 0;
    int32_t *pair_sorted = nullptr;     // [n_m2l] pair index (target order), sorted by translation key
    int32_t *chunk_begin = nullptr;     // [n_chunks + 1] ranges of pair_sorted, one key per chunk
    int32_t *chunk_trans = nullptr;     // [n_chunks] translation of each chunk
    uint64_t *trans_key = nullptr;      // [n_trans]
    cplx<double> *table64 = nullptr;    // [n_trans][(q+1)^2] full irregular tables
    cplx<float> *table32 = nullptr;
    // parent <-> child: the child centre sits at (+-1/2, +-1/2, +-1/2) parent
    // half-sizes from the parent centre; regular tables of the 8 offsets
    int8_t *box_oct = nullptr;          // [nbox] octant of each box in its parent (x<<2 | y<<1 | z)
    cplx<double> *oct64 = nullptr;      // [8][(p_max+1)^2]
    cplx<float> *oct32 = nullptr;
    // M2M and L2L as real linear maps of the stored coefficients (m >= 0, real
    // and imaginary parts interleaved): one D x D matrix per octant at p_max,
    // D = 2 ncoef(p_max), stored input-major ([o][k][r]); order p uses the
    // leading 2 ncoef(p) block
    int op_dim = 0;
    double *m2m64 = nullptr, *l2l64 = nullptr;
    float *m2m32 = nullptr, *l2l32 = nullptr;
    // the boxes of each level >= 1 grouped by octant, in tiles of at most
    // 16 / nch boxes: level l owns tiles [tile_begin[l], tile_begin[l + 1])
    std::vector<int> tile_begin;
    int4 *tiles = nullptr;              // octant, first entry of level_list, count, 0
    int32_t *level_list = nullptr;
    // boxes with children, by level: level l owns [par_begin[l], par_begin[l + 1])
    std::vector<int> par_begin;
    int32_t *parents = nullptr;
    // coarsest levels holding an M2L source / target: M2M into levels above
    // the first and L2L out of levels above the second carry nothing
    int lmin_src = 0, lmin_tgt = 0;
    int32_t *leaf_rec = nullptr;        // [nleaf][LEAF_REC]: see LEAF_REC
    int32_t *reduce_order = nullptr;    // [nbox] target boxes of the M2L sum, most pairs first
    void *Z = nullptr;                  // [nbox][nch][ncoef(p_max)] complex FP64: per-child M2M terms
    // stored FP64 pass-1 operators (m2l_stored): per translation, row tiles
    // rt < ops_nrt of 16 rows, column steps kt < ops_k4 of 4 inputs, 64
    // values per (rt, kt) in the matrix-core lane order
    double *ops64 = nullptr;
    int ops_nrt = 0, ops_k4 = 0;
    int64_t ops_bytes = 0;
    // M2L by rotation (m2l_stored = 2, rotations.cpp): per direction (an
    // integer offset reduced by its gcd) the folded forward and backward
    // rotations of every degree <= p_max in matrix-core lane order (rot_per
    // values per direction and kind), FP64 and FP32.  The chunks are taken in
    // the order of their directions, so that the chunks sharing a direction's
    // tables run together on one XCD; per position in that order: rot_hdr =
    // {direction, eT | eS << 8, columns, 0} and rot_dist = |D| 2^-e (in units
    // of the larger half-size), per column rot_cols = {source box x channels
    // + channel, pair x channels + channel} ({-1, -1} past the chunk), and for
    // Stokes per pair rot_gc = c_S - c_T
    int n_dirs = 0;
    int64_t rot_per = 0, rot_bytes = 0;
    int4 *rot_hdr = nullptr;
    int2 *rot_cols = nullptr;
    double *rot_dist = nullptr, *rot_gc = nullptr;
    double *rot64_f = nullptr, *rot64_b = nullptr;
    float *rot32_f = nullptr, *rot32_b = nullptr;
};
// orders from which the rotation M2L replaces the direct one (m2l_stored = 2)
constexpr int ROT_MIN_P = 7;
// orders up to which L2P (where the downward pass is not fused) evaluates the
// far field without waiting for the near field, and a combine joins the two
constexpr int L2P_FAR_MAX_P = 7;

// The regular near field stored as a block-sparse matrix (nearfield.hip): per
// P2P unit (targets [tb, te) of one leaf), one dense block per source leaf of
// its P2P list, n_u x n_S entries stored source-major ([j][i], Stokes
// [j][a*3+b][i]), the target's own panel zero (it enters through the
// correction).  FP64 values and an FP32 copy rounded from them.
struct NearBlock {
    int32_t j0, ns;  // first source panel (sorted order), source panels
    int64_t off;     // first value
};
struct NearMatrix {
    int64_t entries = 0;            // panel pairs
    int64_t nblk = 0;
    int32_t *blk_ptr = nullptr;     // [n_unit + 1]
    NearBlock *blk = nullptr;       // [nblk]
    double *v64 = nullptr;
    float *v32 = nullptr;
    double *xs = nullptr;           // [n] the mat-vec input in sorted panel order
    int64_t folded = 0;             // corrections added into the stored blocks
    Correction rest;                // corrections whose pair has no stored block
};

// GMRES workspace (krylov.hip): one per context from its allocator, or a
// view of the library's static scratch array (the allocation-free solve)
struct KrylovWork {
    int m = 0;
    int64_t n = 0;
    int nb = 0;              // row blocks of the dot-product kernels
    int rpt = 1;             // rows per thread in those blocks
    double *V = nullptr;     // [m+1][n]
    double *w = nullptr;     // [n]
    double *r = nullptr;     // [n]
    double *part1 = nullptr; // [m+1][nb] per-block partials of the first Gram-Schmidt pass
    double *part2 = nullptr; // [m+1][nb] the second pass
    double *partn = nullptr; // [nb] |w|^2
    double *y = nullptr;     // [m+1] least-squares solution, copied from hcol
    // Hessenberg column in pinned, device-mapped host memory, written by the
    // kernels directly: h1[0..k], |w|^2 at k + 1, h2 at m + 2 + j, |b|^2 at
    // 2 (m + 2); the least-squares solution y (host-written) after it
    double *hcol = nullptr;      // host view, [hcol_len(m)]
    const PinnedProvider *hcol_src = nullptr;
    double *hcol_dev = nullptr;  // the same memory, device view
    hipEvent_t ev_h = nullptr;   // the column of the last step is complete
    bool owned = true;           // V ... hcol, ev_h belong to this workspace
    DevArena arena;
};
inline int64_t hcol_len(int m) { return 2 * (int64_t)(m + 2) + 1 + (m + 1); }
// row blocks and rows per thread of the Arnoldi kernels for n rows
void krylov_blocks(int64_t n, int *nb, int *rpt);

}  // namespace fmmbem

#include <chrono>

struct fmmbem_ctx {
    int kernel = FMMBEM_LAPLACE_SL;
    fmmbem_params prm{};
    int device = 0;
    int64_t nt = 0, n = 0, nsrc = 0;
    int nch = 1;  // expansion channels: 1 Laplace, 4 Stokes
    fmmbem::DevArena arena;
    fmmbem::Tree tree;
    fmmbem::Geometry geo;
    fmmbem::Correction corr;
    // per-mat-vec workspace
    void *charges = nullptr;   // [nsrc] packed sources (position + charges) of the current mat-vec
    void *Y = nullptr;         // [n_m2l][nch][NC(p)] per-pair M2L results
    fmmbem::M2LPlan m2l;
    void *M = nullptr;         // [nbox][nch][NC(p_max)] complex Real
    void *L = nullptr;         // same
    double *y_near = nullptr;  // [n] sorted order (P2P + far field, in kernel units)
    double *y_far = nullptr;   // [n]
    double *y_corr = nullptr;  // [n] sorted order: the correction's product S x of the current mat-vec
    fmmbem::Timing timing;
    fmmbem::KrylovWork *kw = nullptr;
    fmmbem::NearMatrix nearm;
    // The near field and the far-field chain of a mat-vec run concurrently on
    // two streams: the near field on the side stream (fork after the charges,
    // join before the combine), or, where it is the longer of the two
    // (near_on_main), the near field on the main stream right after the
    // charges and the far chain on the side stream, joined before the combine
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool side_pending = false;  // work on the side stream that the main stream has not joined yet (ev_join marks its end)
    bool corr_on_near = false;  // the correction product of the pending near field runs behind it on the side stream
    // charges already launched for this input and precision ahead of the
    // mat-vec that will use them, with the upward pass of order spec_up_p
    // (-1: none; see prefetch_charges)
    const double *spec_x = nullptr;
    int spec_prec = -1;
    int spec_up_p = -1;
    bool spec_near = false;  // the near field of those charges already launched
    bool spec_swap = false;  // the prefetched mat-vec runs its near field on the main stream (near_on_main)
    // Hessenberg column of fmmbem_solve_ctx_static (pinned, device-mapped,
    // made at build for restarts up to FMMBEM_STATIC_MAX_RESTART) and its event
    double *hcol_s = nullptr, *hcol_s_dev = nullptr;
    const fmmbem::PinnedProvider *hcol_s_src = nullptr;
    hipEvent_t ev_h_s = nullptr;
};

namespace fmmbem {

struct Sched {
    int p;
    int prec;
};

// GMRES(m) as a state machine so that a request loop can interleave solves:
// start(); while (!done) { enqueue_step(); complete_step(); }
// enqueue_step only enqueues device work on the solve's stream (mat-vec,
// CGS2, the Hessenberg column into pinned memory); complete_step waits for it
// and applies the Givens update on the host.  The host arrays (Hessenberg
// matrix, rotations, right-hand side) come from hostw when given (4 m + 2 +
// (m + 1) m doubles), else from the state's own vector; the histories go
// straight to rep's caller-owned arrays.
struct GmresState {
    fmmbem_ctx *ctx;
    const double *b;
    double *x;
    fmmbem_schedule s;
    double tol;
    hipStream_t st;
    KrylovWork *kw = nullptr;
    fmmbem_report *rep = nullptr;
    std::vector<double> host_own;
    double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *yv = nullptr;
    double *hbuf = nullptr;     // kw->hcol
    hipEvent_t ev_h = nullptr;  // kw->ev_h
    int it = 0, restarts = 0, converged = 0, k = 0, fallbacks = 0, stalls = 0;
    int p_floor = 0;  // raised by a stalled cycle: no later order falls below it
    int64_t matvecs = 0;
    double bnorm = 0, beta = 0, rel = 1, true_rel = 1, rho_prev = 1;
    double rho_prev2 = -1;  // the residual before rho_prev, < 0 if none
    bool done = false;
    bool bnorm_known = true;  // false from the start until the first column is read
    bool fp64_only = false;   // after a non-finite residual: every later mat-vec in FP64
    Sched cur{0, 0};
    double t_stage0[FMMBEM_N_STAGES] = {0};  // the context's stage times at the start
    std::chrono::steady_clock::time_point t0, t1;

    static size_t host_doubles(int m) { return 4 * (size_t)m + 2 + (size_t)(m + 1) * m; }
    GmresState(fmmbem_ctx *c, const double *b, double tol, const fmmbem_schedule *s, double *x, hipStream_t st,
               fmmbem_report *rep = nullptr, KrylovWork *kw_given = nullptr, double *hostw = nullptr);
    ~GmresState();
    GmresState(const GmresState &) = delete;
    GmresState &operator=(const GmresState &) = delete;
    void start();
    void enqueue_step();
    void complete_step();
    void fill_report(fmmbem_report *rep) const;

  private:
    void begin_cycle();
    void end_cycle();
    void record(int p, int prec, double r);
    void drain_prefetch();
};

void build_geometry_and_tree(fmmbem_ctx *ctx, const fmmbem_mesh *mesh, hipStream_t st);
void build_correction(fmmbem_ctx *ctx, hipStream_t st);
// C.val32 from C.val (the correction that the mat-vecs read)
void correction_fp32(fmmbem_ctx *ctx, Correction &C, hipStream_t st);
void build_translations(fmmbem_ctx *ctx, hipStream_t st);
void run_matvec(fmmbem_ctx *ctx, int p, int prec, const double *x, double *y, hipStream_t st);
// launch the charges of a mat-vec on x at precision prec ahead of time (the
// input written there first as w / |w| from the partial sums nz.partn when
// they are given: see k_charges; the
// next run_matvec with the same x and prec uses them and starts the near field
// from them), then optionally the upward pass (P2M, M2M) of order p_up, whose
// multipoles that run_matvec uses when its order is <= p_up
// (near_main: the mat-vec will run its near field on the main stream st and
// its upward pass and far chain on the side stream)
void prefetch_charges(fmmbem_ctx *ctx, int prec, const double *x, hipStream_t st, const NormIn &nz = NormIn{},
                      bool near_main = false);
void prefetch_up(fmmbem_ctx *ctx, int prec, int p_up, hipStream_t st);
// launch the near field of the prefetched charges now (on the side stream, or
// on st for near_main)
void prefetch_near(fmmbem_ctx *ctx, hipStream_t st);
// whether a mat-vec of order p and precision prec runs its near field on the
// main stream and its far chain on the side stream: FP32 Stokes with the
// near field on the fly at the orders where its L2P evaluates the far field
// alone (the near field is then the longer branch)
bool near_on_main(const fmmbem_ctx *ctx, int p, int prec);
// stored near field (nearfield.hip): assemble at build; one product on
// stream st of the input in sorted order (nearm.xs, written by the charges)
void build_near_matrix(fmmbem_ctx *ctx, hipStream_t st);
// stored FP64 M2L operators (fmm.hip), after build_translations
void build_m2l_operators(fmmbem_ctx *ctx, hipStream_t st);
void launch_near_stored(fmmbem_ctx *ctx, int prec, hipStream_t st);
int run_solve(fmmbem_ctx *ctx, const double *b, double tol, const fmmbem_schedule *s, double *x,
              fmmbem_report *rep, hipStream_t st);
// x[0..n) = 0 by a kernel (no memset node in a caller's capture)
void fill_zero(double *x, int64_t n, hipStream_t st);
void free_krylov(fmmbem_ctx *ctx);
// fmmbem_destroy; without sync_device the caller has synchronised every
// stream that used the context (the request loop, which must not drain the
// device while other requests run)
void destroy_context(fmmbem_ctx *ctx, bool sync_device);
// allocate the context's Krylov workspace for GMRES(m) now (a solve would on
// its first call)
void reserve_krylov(fmmbem_ctx *ctx, int m);
// GMRES with the Krylov workspace in the library's static device array
// (fmmbem_solve_ctx_static); no device or host memory is allocated
int run_solve_static(fmmbem_ctx *ctx, const double *b, double tol, const fmmbem_schedule *s, double *x,
                     fmmbem_report *rep, hipStream_t st);
// timing helpers (api.hip); timing_resolve reads every pending event pair
void timing_resolve(Timing &T);
void stage_begin(fmmbem_ctx *ctx, int stage, hipStream_t st, hipEvent_t *ev);
void stage_end(fmmbem_ctx *ctx, int stage, hipStream_t st, hipEvent_t ev, double flops = 0.0);
// rules (rules.cpp): Gauss-Legendre by Golub-Welsch, near rule tables
void gauss_legendre_gw(int n, double *x, double *w);
// rotation tables of the M2L by rotation (rotations.cpp): values per
// direction and kind at order p, and the tables of the given integer directions
int64_t rot_tile_values(int p);
void rotation_tables(const std::vector<std::array<int64_t, 3>> &dirs, int p, std::vector<double> &fwd,
                     std::vector<double> &back);
void near_rule_table(int n1d, double *bary, double *w);
void set_last_error(const std::string &m);
inline int grid_for(int64_t n, int block) { return (int)((n + block - 1) / block); }
}  // namespace fmmbem
