// internal.h -- data structures shared by the host set-up code, the kernels
// and the C-ABI layer of the gfx950 two-level solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/iga2l.h"

namespace iga2l {

constexpr int kMaxDim = 3;
// the V-cycle hierarchy stops at the first level with at most this many
// unknowns; that level is solved exactly
constexpr int64_t kCoarsestMax = 512;
constexpr int kMaxP = 8;

// -------------------------------------------------------------- errors --
void set_error(const std::string &msg);

struct Error {
    int code;
    std::string msg;
};

#define IGA2L_HIP(call)                                                                \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::iga2l::Error{IGA2L_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define IGA2L_REQUIRE(cond, code, msg)                                                 \
    do {                                                                               \
        if (!(cond)) throw ::iga2l::Error{(code), (msg)};                              \
    } while (0)

// --------------------------------------------------------- device buffer --
// Owning device allocation; freed with the problem.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    void alloc(size_t nbytes);
    void free();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
    ~DevBuf() { free(); }
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ptr(o.ptr), bytes(o.bytes) {
        o.ptr = nullptr;
        o.bytes = 0;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            free();
            ptr = o.ptr;
            bytes = o.bytes;
            o.ptr = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
};

// ---------------------------------------------------------- grid shapes --
// A tensor grid of n1 points per direction in dim directions, x fastest.
struct Grid {
    int dim = 2;
    int n1 = 0;
    int64_t n = 0;
};

// Banded operator with radius q stored in symmetric "upper-diagonal" form:
// for each offset o in [-q,q]^d whose lexicographic (z,y,x) sign is >= 0
// (Wh = ((2q+1)^d + 1) / 2 of them, the centre first) an array of the entries
// A[i][i+o] over the padded grid (n1 + 2q per direction, zero padding), so
// that A[i][i-o] = A[i-o][i] is read at the shifted padded position.
struct SymDia {
    int q = 0;
    int W = 0, Wh = 0;
    int pitch[kMaxDim] = {1, 0, 0};  // padded strides
    int64_t npad = 0;                // padded length of one diagonal
    DevBuf v64, v32;                 // [Wh][npad]
};

// One level of the degree-1 V-cycle hierarchy: full 3^d stencil by offset,
// stored [3^d][n] (structure of arrays), and the reciprocal diagonal.
struct Level {
    Grid g;
    DevBuf S64, S32, invd64, invd32;
    DevBuf Zinv64, Zinv32;       // coarsest level only: dense inverse [n][n]
    DevBuf e[2], rhs, res;       // working vectors, sized for FP64 (FP32 reuses them)
    bool cst = false;            // translation-invariant stencil (interior row everywhere)
};

// Level descriptor handed to the V-cycle kernels (by value or in a device array).
template <class T>
struct LevelDev {
    int n1;
    int cst;          // 1: use c[] / cinv instead of S / invd
    int64_t n;
    const T *S;       // [3^d][n]
    const T *invd;    // [n]
    const T *Zinv;    // coarsest level: dense inverse [n][n], else null
    T c[27];          // interior stencil (cst only)
    T cinv;           // 1 / centre coefficient (cst only)
};

struct Problem {
    int device = 0;
    int dim = 2, p = 3, m = 0;
    Grid fine, coarse;      // fine: n1 = m+p-2; coarse: n1 = m-1 (degree 1)
    int64_t ne = 0;
    bool kappa_one = true;
    // geometry: the unit square (B-splines) or the quarter annulus of radii
    // r_in < r_out (NURBS, Section 5.2).  For the annulus the operator and the
    // transfers are tensor sums/products of direction-dependent 1-D factors:
    // K1, M1, R1 hold the angular (x) direction, K1y, M1y, R1y the radial (y)
    int geometry = 0;   // kGeomSquare or kGeomAnnulus
    double r_in = 0.0, r_out = 0.0;
    std::vector<double> K1y, M1y, R1y;
    std::vector<double> kappa;

    // host copies of the 1-D factors (per direction identical)
    std::vector<double> K1, M1;   // [n1][2p+1], interior rows, offset j-i+p
    int plow = 1;                 // degree of the coarse space (1 or 2)
    std::vector<double> R1;       // [n1c][p+plow+1], coarse row I, fine column I-plow+a
    std::vector<double> Mx1;      // the same without the lumped scaling: Mmix1
    std::vector<std::vector<double>> Ke, Me;  // element matrices [m][(p+1)^2]

    SymDia A;                     // fine stiffness
    DevBuf R1d64, R1d32;          // restriction factor on the device
    DevBuf R1yd64, R1yd32;        // the radial factor of the annulus (empty otherwise: R1 serves every axis)
    int64_t fdm_axis_stride = 0;  // fast diagonalisation: 0 one matrix for every axis, n1c^2 one per axis
    DevBuf Ke_d, Me_d;            // 1-D element matrices (FP64) for the gradient kernel
    DevBuf kappa_d;

    // Schwarz blocks
    int bw = 0, bd = 0;           // block width, b^d
    int ncls1 = 0;                // classes per direction (1-D block classes)
    bool shared_inverses = false; // kappa = 1: one inverse per class, else one per DOF
    DevBuf cls_d;                 // [n1] int: 1-D class of a block centre
    DevBuf Inv64, Inv32;          // [nslots][bd][bd]
    int64_t nslots = 0;
    bool blocks_ready = false;
    bool fp32_ready = false;
    // lexicographic schedule: hyperplane steps
    std::vector<int> lex_off;     // host [nsteps+1]
    DevBuf lex_blocks;            // int [n]
    DevBuf lex_off_d;             // the step offsets on the device
    int lex_maxcnt = 0;           // most blocks in one step

    // coarse
    std::vector<Level> levels;    // V-cycle hierarchy, level 0 = A_1 on the same knots
    std::vector<LevelDev<double>> levhost64;
    std::vector<LevelDev<float>> levhost32;
    DevBuf levdev64, levdev32;    // the same descriptors on the device
    size_t vc_bottom64 = 0, vc_bottom32 = 0;  // first level run by the one-workgroup kernel
    bool vcycle_ready = false;
    DevBuf dst_S, dst_mu;         // DST-I matrix [n1c][n1c], eigenvalues [n_c]
    DevBuf coarse_inv64;          // variable kappa: A_1^{-1} [n_c][n_c] (exact coarse solve), else empty
    bool direct_ready = false;
    // exact (not lumped) transfers: the degree-1 mass matrix M_1 is diagonalised
    // by the same DST-I; dstM_mu holds its eigenvalues (products of the 1-D
    // ones), Mx64/Mx32 the unlumped 1-D factor Mmix1 [n1c][p+2]
    DevBuf dstM_S, dstM_mu, Mx64, Mx32, ctmp2;
    // degree-2 coarse space (kappa = 1): fast diagonalisation, forward V^T and
    // backward V per axis; dst_mu then holds the eigenvalue sums, dstM_mu ones
    DevBuf fdm_Vt, fdm_V;
    bool mass_ready = false;
    // aggressive coarsening (degree 1 on 2h): exact 2h solve by the DST-I of
    // level 1 of the V-cycle hierarchy (kappa = 1, m even)
    DevBuf dst2_S, dst2_mu, agg64, agg32;
    bool agg_direct_ready = false;
    // while a call runs: apply the exact transfers (else the lumped ones)
    bool transfer_exact = false;
    bool lumped_default = true;   // transfers of iga2l_restrict / iga2l_prolong (last set-up)
    double t_setup_ms = 0.0;      // host wall time of assembly and set-up so far

    // workspaces
    DevBuf r64;                   // fine residual FP64
    DevBuf ework[2];              // fine correction ping-pong (FP64-sized)
    DevBuf rhs_w;                 // fine right-hand side in working precision
    DevBuf dfine;                 // fine defect in working precision
    DevBuf dc, ec, ctmp;          // coarse vectors (FP64-sized)
    DevBuf dc64, ec64;            // FP64 coarse vectors of the exact solve in mixed mode
    DevBuf partial;               // per-workgroup partial sums (FP64)
    int hist_cap = 0;             // cycles of history held after the flags in scal
    const int *skip = nullptr;    // while a solve runs: flags (kernels return at once when set)
    void *host_status = nullptr;  // pinned host copy of flags + hist
    int expected_cycles = 8;      // cycles of the last solve: size of the first batch
    DevBuf cs64, cs32;            // interior stencil of kappa = 1 rows, (2p+1)^d (empty otherwise)
    DevBuf kron64, kron32;        // kappa = 1, 3-D: K1 then M1, [n1][2p+1] each (empty otherwise)
    DevBuf cf64, cf32;            // kappa = 1: interior row of K1 then of M1, 2 (2p+1) (empty otherwise)
    DevBuf fac64, fac32;          // kappa = 1, 2-D: K1, M1, K1, M1, [n1][2p+1] each (empty otherwise)
    DevBuf fac2d64, fac2d32;      // annulus: rows of K1, M1, K1y, M1y, [n1][2p+1] each (empty otherwise)
    int ulo = 1, uhi = 0;         // rows with all coordinates in [ulo, uhi] carry that stencil
    DevBuf scal;                  // status block: kScalCount doubles, kFlagCount ints, hist_cap doubles
    DevBuf lam_tmp;               // adjoint workspace
    int npartial = 0;

    ~Problem() {
        if (host_status) (void)hipHostFree(host_status);
    }

    // tuning knobs (numerics-neutral): Schwarz tile in blocks, per working
    // precision ([0] FP64, [1] FP32); 2-D shapes are chosen by the autotuner
    int tile_bx[2] = {4, 4}, tile_by[2] = {4, 4}, tile_bz = 1;
    bool tuned[2] = {false, false};

    // identifies the device layout (buffers, levels, set-up state); renewed
    // whenever it changes, never reused, so cached batch plans can tell
    // whether they still describe this problem
    uint64_t layout_id = 0;
};

uint64_t next_layout_id();

// device scalar slots in Problem::scal (doubles)
enum { kScalNorm = 0, kScalSigma = 1, kScalInvSigma = 2, kScalR0 = 3, kScalTol = 4, kScalMaxCycles = 5, kScalCount = 8 };
// device int slots in Problem::flags: stop flag, cycles done, status (0 running/converged, 1 max cycles, 2 numeric)
enum { kFlagDone = 0, kFlagIter = 1, kFlagStatus = 2, kFlagCount = 4 };

// Workgroups are dealt to the XCDs (each with its own L2) round-robin by
// linear id.  xcd_tile_2d relabels a 2-D grid of tiles so that the workgroups
// one XCD runs cover a contiguous band of tiles in row-major order: halos
// shared by neighbouring tiles are then re-read from the same L2.  The map is
// a bijection of the tile set; results do not depend on it.
constexpr int kNumXcd = 8;
__host__ __device__ __forceinline__ void xcd_relabel(int b, int ntx, int nb, int &bx, int &by) {
    const int x = b % kNumXcd, k = b / kNumXcd;
    const int q = nb / kNumXcd, r = nb % kNumXcd;
    const int L = x * q + (x < r ? x : r) + k;
    bx = L % ntx;
    by = L / ntx;
}
__device__ __forceinline__ void xcd_tile_2d(int &bx, int &by) {
    xcd_relabel(int(blockIdx.y * gridDim.x + blockIdx.x), int(gridDim.x), int(gridDim.x * gridDim.y), bx, by);
}

// LDS staging of a window of a grid: dst[h] = get(h) for h < nh, thread t
// taking h = t, t + blockDim, ...  Each thread issues U loads before its
// first LDS store, so U memory round trips overlap instead of following one
// another (a plain strided loop waits for every load before the next).
template <int U, class T, class Get>
__device__ __forceinline__ void stage_lds(T *dst, int nh, Get get) {
    const int nt = int(blockDim.x);
    for (int base = int(threadIdx.x); base < nh; base += U * nt) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int hh = base + u * nt;
            v[u] = hh < nh ? get(hh) : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int hh = base + u * nt;
            if (hh < nh) dst[hh] = v[u];
        }
    }
}

// block classes of the Schwarz inverses, as the kernels compute them: the
// number L of boundary classes on each side with shared inverses, -1 when
// every position has its own inverse (must match host_block_classes)
inline int class_split(const Problem &P) { return P.shared_inverses ? (P.ncls1 - 1) / 2 : -1; }

// 1-D class of a block centre j (the index of its inverse along one
// direction): with shared inverses (kappa = 1, L = p-1+h_b) the first and
// last L positions have their own classes and all others share class L;
// otherwise (L < 0) every position is its own class.  Computed instead of
// looked up, so the inverse rows can be loaded together with the halo.
__device__ __forceinline__ int block_class(int j, int n1, int L) {
    if (L < 0) return j;
    return j < L ? j : (j > n1 - 1 - L ? L + 1 + (j - (n1 - L)) : L);
}

// views into the status block
inline int *dev_flags(const Problem &P) { return reinterpret_cast<int *>(P.scal.as<double>() + kScalCount); }
inline double *dev_hist(const Problem &P) { return P.scal.as<double>() + kScalCount + kFlagCount / 2; }
inline size_t status_bytes(int hist_cap) { return sizeof(double) * (kScalCount + kFlagCount / 2 + hist_cap); }

// ------------------------------------------------------ batched launches --
// A batched launch runs one step of the cycle for many independent 2-D
// problems at once: workgroup w handles tile map[w].y of problem map[w].x,
// with that problem's operands read from a device table.  The arithmetic of
// every tile is that of the single-problem kernel, so batched and single
// solves agree bitwise.
enum VecRole { kVecU, kVecB, kVecR64, kVecE0, kVecE1, kVecRhsW, kVecDFine, kVecDC, kVecEC, kVecCount };

struct BatchProb {
    const void *val[2], *inv[2], *cs[2], *R1[2];   // [0] FP64, [1] FP32 (null if not set up)
    const void *fac[2];                            // the Schwarz colour's 1-D factor rows (colour_factor_rows)
    const int *cls;
    int clsL;                                      // block classes: L of shared inverses, -1 = one per position
    int64_t npad;
    int pitch1, n1, n1c, p, ncls1, ulo, uhi;
    int hist_cap;
    double *scal, *partial, *hist;
    int *flags;                                    // also the stop flag of every kernel
    void *vec[kVecCount];
    int res_ntx, res_nty;                          // residual tiles (64 x 4 points)
    int col_ntx, col_nty;                          // colour tiles, a grid covering every colour
    int tr_cx, tr_cy, tr_ntx, tr_nty;              // restriction tiles (coarse points)
    int pr_tx, pr_ty, pr_ntx, pr_nty;              // prolongation tiles (fine points)
};

// level l (above the one-workgroup tail) of one problem's V-cycle
template <class T>
struct BatchLevel {
    LevelDev<T> L;
    const T *rhs;      // right-hand side of the level
    T *e_pre;          // pre-smoothed iterate
    T *rc;             // restricted residual = right-hand side of level l+1
    const T *ecl;      // correction of level l+1
    T *e_out;          // result of the level
    int n1c;           // points per direction of level l+1
    int ntx, nty;      // 32 x 8 tiles
    const int *skip;
};

// one problem's tail of the V-cycle (one workgroup)
template <class T>
struct BatchBottom {
    const LevelDev<T> *levels;   // first entry = first level of the tail
    int nlev;
    const T *rhs;
    T *e;
    const int *skip;
};

void launch_norm_finalize_batch(const BatchProb *bp, int nprob, bool scale_fp32, bool book, hipStream_t s);
void launch_solve_init_batch(const BatchProb *bp, int nprob, double tol, int max_cycles, hipStream_t s);
template <class T>
void launch_colour_batch(const BatchProb *bp, const int2 *map, int nwg, int p, int bw, int nbx, int nby, int cx,
                         int cy, int S, int role_src, int role_dst, int role_rhs, bool x_zero, bool fuse,
                         hipStream_t s, bool use_skip = true);
template <class T>
void launch_residual_batch_dispatch(int p, const BatchProb *bp, const int2 *map, int nwg, int role_x, int role_b,
                                    int role_r, bool norm, bool use_skip, hipStream_t s);
template <class T>
void launch_restrict_batch(const BatchProb *bp, const int2 *map, int nwg, size_t shm, int role_f, int role_c,
                           hipStream_t s);
template <class T>
void launch_prolong_update_batch(const BatchProb *bp, const int2 *map, int nwg, size_t shm, int role_c, int role_e,
                                 bool scaled, hipStream_t s);
size_t restrict2d_lds(int p, int cx, int cy, size_t elem);
size_t prolong2d_lds(int p, int tx, int ty, size_t elem);
void transfer_tile_2d(int64_t n1, int &tx, int &ty);
template <class T>
void launch_rb_multi2_batch(const BatchLevel<T> *bl, const int2 *map, int nwg, int nu, bool restrict_, bool zero_src,
                            hipStream_t s);
template <class T>
void launch_vcycle_bottom_batch(const BatchBottom<T> *bb, int nprob, size_t shm, int nu1, int nu2, hipStream_t s);
size_t colour_lds(int p, int S, int nbx, int nby, size_t elem, bool factor_rows);
// the 1-D factor rows from which the 2-D Schwarz colour forms every operator
// row, and the tiled residual the rows of its wavefronts next to the boundary
// (rows of Kx, Mx, Ky, My, [n1][2p+1] each): the quarter annulus's, and a
// kappa = 1 square's on grids below the streamed sizes; null: the stencil and
// the stored diagonals
const void *colour_factor_rows(const Problem &P, bool fp64);
void colour_tile_clamp(int S, int &nbx, int &nby);

// grows the status block so that it holds cap cycles of history
void ensure_history(Problem &P, int cap);
// the batched solve handles these problems and options (2-D, coloured
// Schwarz, fused V-cycle, below 2^20 unknowns each, one device)
bool batch_supported(Problem *const *probs, int nprob, const iga2l_opts &o);
// worst / msg: the first non-converged (or numerically failed) problem
void solve_batch_fused(Problem *const *probs, int nprob, const double *const *b, double *const *u,
                       const iga2l_opts &o, iga2l_info *infos, hipStream_t s, int &worst, std::string &msg);

// ------------------------------------------------------------ host set-up --
enum { kGeomSquare = 0, kGeomAnnulus = 1 };
void host_assemble(Problem &P);                 // 1-D factors, DIA, transfers, kappa
void host_build_levels(Problem &P);             // V-cycle hierarchy (Galerkin)
void host_build_dst(Problem &P);                // exact coarse solver
// largest coarse space with variable kappa solved exactly (dense inverse)
constexpr int64_t kCoarseInvMax = 4096;
void host_build_mass(Problem &P);               // exact M_low^{-1} transfers (DST-I / fast diagonalisation)
void host_transfer_factors(Problem &P, int plow);  // 1-D transfer factors, coarse grid of degree plow
void host_coarse_workspaces(Problem &P);        // coarse vectors sized by the coarse grid
void host_set_coarse_degree(Problem &P, int plow);
void host_build_fdm(Problem &P);                // exact degree-2 coarse solve (kappa = 1)
void host_build_agg_direct(Problem &P);         // exact 2h solve of aggressive coarsening
void host_block_classes(Problem &P, std::vector<int> &cls1, std::vector<int64_t> &reps);
void host_lex_schedule(Problem &P);

// ------------------------------------------------------------ launchers --
// fine level
void launch_block_inverse(Problem &P, const std::vector<int64_t> &reps, hipStream_t s);
// r = b - A u in FP64; with_norm: also ||r||_2 and the FP32 scaling into P.scal;
// book: also the device-side convergence test after a cycle (P.flags, P.hist)
void launch_residual64(const Problem &P, const double *u, const double *b, double *r, bool with_norm,
                       bool scale_fp32, bool book, hipStream_t s);
template <class T>
void launch_defect(const Problem &P, const T *e, const T *rhs, T *d, hipStream_t s);
void launch_solve_init(const Problem &P, double tol, int max_cycles, hipStream_t s);
int64_t residual_workgroups(const Problem &P);   // partial sums written by the FP64 residual
// one colour of the Schwarz sweep; r64/rhs_out: fused FP32 cast of the residual
// (first colour of an FP32 correction sweep only)
template <class T>
void launch_colour_step(const Problem &P, int cx, int cy, int cz, int s_period, const T *x_src, T *x_dst,
                        const T *rhs, bool x_zero, hipStream_t s, const double *r64 = nullptr, T *rhs_out = nullptr);
void launch_lex_step(const Problem &P, int step, double *u, const double *b, hipStream_t s);
// the whole lexicographic sweep in one workgroup (iterate in LDS) when it fits
bool lex_sweep_fits(const Problem &P);
void launch_lex_sweep(const Problem &P, double *u, const double *b, hipStream_t s);
// times the coloured Schwarz kernel for candidate tile shapes on the problem's
// own workspaces (2-D) and keeps the fastest in P.tile_bx / P.tile_by
template <class T>
void autotune_colour_tile(Problem &P, int S, hipStream_t s);
// IGA2L_TUNE_LOG=1 in the environment: the autotuners print their timings to stderr
bool tune_log();
// candidate tile shapes (blocks per tile in x, y) for a colour period S
std::vector<std::pair<int, int>> colour_tile_candidates(int S, int n1);
template <class T>
void launch_cast_scale(const Problem &P, const double *r64, T *rhs, hipStream_t s);
// 3-D kappa = 1 by sum factorisation (kernels_3d.hip): the Schwarz colour with
// colour period 3 and 3x3x3 blocks (shared inverse applied by MFMA) and the residual
bool colour3d_sf_ok(const Problem &P, int S);
bool residual3d_sf_ok(const Problem &P);
int64_t residual3d_sf_workgroups(const Problem &P);
template <class T>
void launch_colour3d_sf(const Problem &P, int cx, int cy, int cz, const T *x_src, T *x_dst, const T *rhs, bool x_zero,
                        const double *r64, T *rhs_out, hipStream_t s);
template <class T, bool NORM>
void launch_residual3d_sf(const Problem &P, const T *x, const T *b, T *r, double *partial, hipStream_t s);
// 2-D kappa = 1 on large grids (kernels_colour2d.hip): one Schwarz colour with
// colour period b, streamed along y (from a zero iterate: tiles of whole
// cells without a halo); false (nothing launched) where it does not apply.
// colour2d_stream_ok: whether it applies to period S.
bool colour2d_stream_ok(const Problem &P, int S);
bool colour2d_stream(const Problem &P, int cx, int cy, int S, const void *x_src, void *x_dst, const void *rhs,
                     bool x_zero, const double *r64, void *rhs_out, bool fp64, hipStream_t s);
// 2-D bandwidth-oriented variants (kernels_2d.hip)
template <class T>
void launch_residual2d(const Problem &P, const T *val, const T *x, const T *b, T *r, double *partial, hipStream_t s);
int64_t residual2d_workgroups(const Problem &P);
template <class T>
void launch_restrict2d(const Problem &P, const T *df, T *dc, hipStream_t s);
template <class T>
void launch_prolong2d(const Problem &P, const T *ec, T *uf, const T *e, double *u64, bool scaled, hipStream_t s);
// transfers
template <class T>
void launch_restrict(const Problem &P, const T *df, T *dc, hipStream_t s);
template <class T>
void launch_prolong_add(const Problem &P, const T *ec, T *uf, hipStream_t s);
template <class T>
void launch_prolong_update(const Problem &P, const T *ec, const T *e, double *u, bool scaled, hipStream_t s);
// coarse
template <class T>
void launch_vcycle(Problem &P, const T *rhs, T *e, int nu1, int nu2, hipStream_t s);
void launch_dst_solve(Problem &P, const double *d, double *e, hipStream_t s);
void dst_apply_2h(Problem &P, const double *d, double *e, double *t1, hipStream_t s);
// x <- M_1^{-1} x in place on the coarse grid (exact transfers), FP64 or FP32
template <class T>
void launch_mass_solve(Problem &P, T *x, hipStream_t s);
// aggressive coarsening: e = P_0 C P_0^T d, C = exact 2h solve or a V-cycle on levels 1..
template <class T>
void launch_coarse_aggressive(Problem &P, const T *d, T *e, bool exact, int nu1, int nu2, hipStream_t s);
int64_t vcycle_bottom_lds(const Problem &P, size_t lb);   // LDS elements of the one-workgroup tail
bool vcycle_bottom_fits(const Problem &P, size_t lb);
void launch_convert(const void *src, void *dst, int64_t n, bool to_fp32, hipStream_t s, const int *skip = nullptr);
void launch_fill_zero(void *x, int64_t n_elems, bool fp32, hipStream_t s, const int *skip);
// gradient
void launch_grad_kappa(const Problem &P, const double *u, const double *lam, double *g, hipStream_t s);
// operator of a variable coefficient (upper diagonals, padded), from P.Ke_d and P.kappa_d
void launch_assemble_dia(Problem &P, hipStream_t s);
// V-cycle hierarchy: degree-1 operator on the fine knots ([3^d][n], from 1-D
// element matrices [m][2][4] and kappa), and one Galerkin coarsening step
void launch_assemble_q1(int dim, const double *KM1, const double *kappa, int m, double *S, hipStream_t s);
void launch_galerkin(int dim, const double *Sf, int nf1, double *Sc, int nc1, hipStream_t s);

}  // namespace iga2l
