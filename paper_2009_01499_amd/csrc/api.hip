// api.hip -- the extern "C" entry points of include/iga2l.h and the two-level
// cycle driver (Algorithm 1 of arXiv:2009.01499 in correction form: FP64
// residual, a correction cycle in working precision from zero, FP64 update).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>

#include "internal.h"

struct iga2l_problem {
    iga2l::Problem P;
};

namespace iga2l {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

void DevBuf::alloc(size_t nbytes) {
    free();
    if (nbytes == 0) nbytes = 8;
    hipError_t e = hipMalloc(&ptr, nbytes);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        throw Error{IGA2L_ENOMEM, "hipMalloc of " + std::to_string(nbytes) + " bytes failed"};
    }
    bytes = nbytes;
}

void DevBuf::free() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

namespace {

template <class F>
int guarded(F &&f) {
    try {
        f();
        g_last_error.clear();
        return IGA2L_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return IGA2L_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return IGA2L_EDEVICE;
    }
}

iga2l_opts effective_opts(const iga2l_opts *o) {
    iga2l_opts r;
    iga2l_default_opts(&r);
    if (o) r = *o;
    return r;
}

void check_opts(const Problem &P, const iga2l_opts &o) {
    IGA2L_REQUIRE(o.ordering == IGA2L_LEX || o.ordering == IGA2L_COLOUR, IGA2L_EINVAL, "unknown ordering");
    IGA2L_REQUIRE(o.coarse == IGA2L_COARSE_DIRECT || o.coarse == IGA2L_COARSE_VCYCLE, IGA2L_EINVAL,
                  "unknown coarse solver");
    IGA2L_REQUIRE(o.precision == IGA2L_FP64 || o.precision == IGA2L_MIXED_FP32, IGA2L_EINVAL, "unknown precision");
    IGA2L_REQUIRE(o.nu1 >= 0 && o.nu2 >= 0 && o.nu1 + o.nu2 <= 64, IGA2L_EINVAL, "bad V-cycle smoothing counts");
    IGA2L_REQUIRE(o.max_cycles >= 0, IGA2L_EINVAL, "max_cycles must be >= 0");
    IGA2L_REQUIRE(o.tol >= 0.0 && std::isfinite(o.tol), IGA2L_EINVAL, "tol must be finite and >= 0");
    IGA2L_REQUIRE(o.fine_post_sweeps >= 0 && o.fine_post_sweeps <= 16, IGA2L_EINVAL, "bad post-sweep count");
    if (P.blocks_ready && o.ordering == IGA2L_COLOUR) {
        const int s = o.colour_period ? o.colour_period : P.bw;
        IGA2L_REQUIRE(s >= P.bw, IGA2L_EINVAL, "colour period must be >= block width");
    }
    IGA2L_REQUIRE(!(o.ordering == IGA2L_LEX && o.precision != IGA2L_FP64), IGA2L_EUNSUPPORTED,
                  "the lexicographic ordering runs in FP64 only");
    IGA2L_REQUIRE(o.lumped == 0 || o.lumped == 1, IGA2L_EINVAL, "lumped must be 0 or 1");
    IGA2L_REQUIRE(o.aggressive == 0 || o.aggressive == 1, IGA2L_EINVAL, "aggressive must be 0 or 1");
    IGA2L_REQUIRE(o.plow == 1 || o.plow == 2, IGA2L_EINVAL, "plow must be 1 or 2");
    IGA2L_REQUIRE(o.plow == 1 || o.plow <= P.p, IGA2L_EINVAL, "plow may not exceed p");
    IGA2L_REQUIRE(o.plow == 1 || (o.coarse == IGA2L_COARSE_DIRECT && !o.aggressive), IGA2L_EUNSUPPORTED,
                  "the degree-2 coarse space is solved exactly (coarse = COARSE_DIRECT, no aggressive coarsening)");
    if (P.geometry == kGeomAnnulus)
        IGA2L_REQUIRE(o.plow == 2 && o.lumped == 1, IGA2L_EUNSUPPORTED,
                      "the annulus uses the degree-2 coarse space (plow = 2) with the lumped transfers");
}

// Applies the exact (not lumped) transfers while a call runs.
struct TransferGuard {
    Problem &P;
    bool old;
    TransferGuard(Problem &p, bool exact) : P(p), old(p.transfer_exact) {
        IGA2L_REQUIRE(!exact || P.mass_ready, IGA2L_EINVAL, "exact transfers not set up (setup_blocks with lumped = 0)");
        P.transfer_exact = exact;
    }
    ~TransferGuard() { P.transfer_exact = old; }
};

void set_device(const Problem &P) { IGA2L_HIP(hipSetDevice(P.device)); }

// one Schwarz sweep on A e = rhs in working precision (COLOUR ordering).
// e_zero: e is zero on entry (its buffer content is ignored).  Returns the
// buffer index (0/1 of P.ework) holding the result; start = buffer holding e.
// r64 != null: the first colour also casts r64/sigma into rhs (FP32 sweeps from zero)
template <class T>
int sweep_colour(const Problem &P, int s_period, T *rhs, int start, bool e_zero, hipStream_t s,
                 const double *r64 = nullptr) {
    const int S = s_period;
    const int ncz = (P.dim == 3) ? S : 1;
    int cur = start;
    bool zero = e_zero;
    for (int cz = 0; cz < ncz; ++cz)
        for (int cy = 0; cy < S; ++cy)
            for (int cx = 0; cx < S; ++cx) {
                const bool fuse = zero && r64;
                launch_colour_step<T>(P, cx, cy, cz, S, P.ework[cur].as<T>(), P.ework[1 - cur].as<T>(), rhs, zero, s,
                                      fuse ? r64 : nullptr, fuse ? rhs : nullptr);
                cur = 1 - cur;
                zero = false;
            }
    return cur;
}

template <class T>
void coarse_solve(Problem &P, const iga2l_opts &o, const T *dc, T *ec, hipStream_t s) {
    if (o.aggressive) {
        launch_coarse_aggressive<T>(P, dc, ec, o.coarse == IGA2L_COARSE_DIRECT, o.nu1, o.nu2, s);
        return;
    }
    if (o.coarse == IGA2L_COARSE_VCYCLE) {
        launch_vcycle<T>(P, dc, ec, o.nu1, o.nu2, s);
        return;
    }
    IGA2L_REQUIRE(P.direct_ready, IGA2L_EINVAL, "exact coarse solver not set up (iga2l_setup_blocks)");
    if constexpr (std::is_same<T, double>::value) {
        launch_dst_solve(P, dc, ec, s);
    } else {
        launch_convert(dc, P.dc64.ptr, P.coarse.n, false, s, P.skip);
        launch_dst_solve(P, P.dc64.as<double>(), P.ec64.as<double>(), s);
        launch_convert(P.ec64.ptr, ec, P.coarse.n, true, s, P.skip);
    }
}

// One correction cycle: expects r64 = b - A u and the scalars written by the
// norm-carrying residual; performs u += sigma * cycle(0; r64 / sigma).
template <class T>
void correction_cycle(Problem &P, const iga2l_opts &o, double *u, hipStream_t s) {
    T *rhs;
    const double *fuse_r64 = nullptr;
    if constexpr (std::is_same<T, double>::value) {
        rhs = P.r64.as<double>();
    } else {
        rhs = P.rhs_w.as<T>();
        if (o.ordering == IGA2L_COLOUR) fuse_r64 = P.r64.as<double>();  // cast inside the first colour
        else launch_cast_scale<T>(P, P.r64.as<double>(), rhs, s);
    }
    int cur = 0;
    if (o.ordering == IGA2L_LEX && P.lex_off.empty()) host_lex_schedule(P);
    if (o.ordering == IGA2L_COLOUR) {
        const int S = o.colour_period ? o.colour_period : P.bw;
        cur = sweep_colour<T>(P, S, rhs, 0, true, s, fuse_r64);
    } else {
        // lexicographic: FP64 only, in place on a zeroed correction
        launch_fill_zero(P.ework[0].ptr, P.fine.n, false, s, P.skip);
        if (lex_sweep_fits(P))
            launch_lex_sweep(P, P.ework[0].as<double>(), P.r64.as<double>(), s);
        else
            for (size_t st = 0; st + 1 < P.lex_off.size(); ++st)
                launch_lex_step(P, int(st), P.ework[0].as<double>(), P.r64.as<double>(), s);
        cur = 0;
    }
    T *e = P.ework[cur].as<T>();
    launch_defect<T>(P, e, rhs, P.dfine.as<T>(), s);
    launch_restrict<T>(P, P.dfine.as<T>(), P.dc.as<T>(), s);
    if (P.transfer_exact) launch_mass_solve<T>(P, P.dc.as<T>(), s);
    coarse_solve<T>(P, o, P.dc.as<T>(), P.ec.as<T>(), s);
    if (P.transfer_exact) launch_mass_solve<T>(P, P.ec.as<T>(), s);
    const bool scaled = !std::is_same<T, double>::value;
    if (o.fine_post_sweeps == 0) {
        launch_prolong_update<T>(P, P.ec.as<T>(), e, u, scaled, s);
        return;
    }
    launch_prolong_add<T>(P, P.ec.as<T>(), e, s);
    for (int k = 0; k < o.fine_post_sweeps; ++k) {
        if (o.ordering == IGA2L_COLOUR) {
            const int S = o.colour_period ? o.colour_period : P.bw;
            cur = sweep_colour<T>(P, S, rhs, cur, false, s);
        } else if (lex_sweep_fits(P)) {
            launch_lex_sweep(P, P.ework[0].as<double>(), P.r64.as<double>(), s);
        } else {
            for (size_t st = 0; st + 1 < P.lex_off.size(); ++st)
                launch_lex_step(P, int(st), P.ework[0].as<double>(), P.r64.as<double>(), s);
        }
    }
    // u += sigma * e: prolongation of a zero coarse vector adds nothing
    launch_fill_zero(P.ctmp.ptr, P.coarse.n, !std::is_same<T, double>::value, s, P.skip);
    launch_prolong_update<T>(P, P.ctmp.as<T>(), P.ework[cur].as<T>(), u, scaled, s);
}

// Keeps P.skip pointing at the device stop flag while a solve enqueues work.
struct SkipGuard {
    Problem &P;
    SkipGuard(Problem &p, const int *f) : P(p) { P.skip = f; }
    ~SkipGuard() { P.skip = nullptr; }
};

}  // namespace

void ensure_history(Problem &P, int cap) {
    if (cap <= P.hist_cap) return;
    DevBuf nb;
    nb.alloc(status_bytes(cap));
    IGA2L_HIP(hipMemset(nb.ptr, 0, status_bytes(cap)));
    IGA2L_HIP(hipMemcpy(nb.ptr, P.scal.ptr, sizeof(double) * kScalCount, hipMemcpyDeviceToDevice));
    P.scal = std::move(nb);
    if (P.host_status) IGA2L_HIP(hipHostFree(P.host_status));
    P.host_status = nullptr;
    IGA2L_HIP(hipHostMalloc(&P.host_status, status_bytes(cap), hipHostMallocDefault));
    P.hist_cap = cap;
    P.layout_id = next_layout_id();
}

namespace {

// Solve loop.  The convergence test runs on the device (the norm-carrying
// residual after each cycle records the history and raises a stop flag that
// every kernel of later cycles obeys), so the host enqueues cycles in batches
// and synchronises once per batch; the first batch has the length of the
// previous solve.  Results are those of stopping exactly at the tolerance.
void solve_impl(Problem &P, const double *b, double *u, const iga2l_opts &o, iga2l_info *info, hipStream_t s) {
    IGA2L_REQUIRE(P.blocks_ready, IGA2L_EINVAL, "iga2l_setup_blocks must run before iga2l_solve");
    IGA2L_REQUIRE(b && u, IGA2L_EINVAL, "null vector");
    const bool fp32 = o.precision == IGA2L_MIXED_FP32;
    IGA2L_REQUIRE(!fp32 || P.fp32_ready, IGA2L_EINVAL, "FP32 data not set up (setup_blocks with MIXED_FP32)");
    IGA2L_REQUIRE(o.plow == P.plow, IGA2L_EINVAL, "coarse degree differs from the last set-up (iga2l_setup_blocks)");
    IGA2L_REQUIRE(o.coarse != IGA2L_COARSE_VCYCLE || P.vcycle_ready, IGA2L_EINVAL, "V-cycle not set up");
    if (o.aggressive)
        IGA2L_REQUIRE(o.coarse != IGA2L_COARSE_DIRECT || P.agg_direct_ready, IGA2L_EINVAL,
                      "exact 2h solve not set up (setup_blocks with aggressive = 1)");
    else
        IGA2L_REQUIRE(o.coarse != IGA2L_COARSE_DIRECT || P.direct_ready, IGA2L_EINVAL, "exact coarse solver not set up");
    TransferGuard tg(P, !o.lumped);
    ensure_history(P, std::max(o.max_cycles, 1));
    auto t0 = std::chrono::steady_clock::now();
    launch_residual64(P, u, b, P.r64.as<double>(), true, fp32, false, s);
    launch_solve_init(P, o.tol, o.max_cycles, s);
    int issued = 0;
    int batch = std::max(1, std::min(P.expected_cycles, o.max_cycles));
    const double *hs = static_cast<const double *>(P.host_status);
    const int *hf = reinterpret_cast<const int *>(hs + kScalCount);
    {
        SkipGuard guard(P, dev_flags(P));
        while (true) {
            for (int j = 0; j < batch && issued < o.max_cycles; ++j, ++issued) {
                if (fp32) correction_cycle<float>(P, o, u, s);
                else correction_cycle<double>(P, o, u, s);
                launch_residual64(P, u, b, P.r64.as<double>(), true, fp32, true, s);
            }
            IGA2L_HIP(hipGetLastError());
            IGA2L_HIP(hipMemcpyAsync(P.host_status, P.scal.ptr, status_bytes(std::min(issued, P.hist_cap)),
                                     hipMemcpyDeviceToHost, s));
            IGA2L_HIP(hipStreamSynchronize(s));
            if (hf[kFlagDone] || issued >= o.max_cycles) break;
            batch = 1;
        }
    }
    const int k = hf[kFlagIter];
    const double r0 = hs[kScalR0];
    const double rel = (k > 0) ? hs[kScalCount + kFlagCount / 2 + k - 1] : (r0 > 0 ? 1.0 : 0.0);
    int status = IGA2L_OK;
    if (hf[kFlagStatus] == 2) status = IGA2L_ENUMERIC;
    else if (hf[kFlagStatus] == 1 || (!hf[kFlagDone] && rel > o.tol)) status = IGA2L_ENOTCONV;
    if (k > 0) P.expected_cycles = k;
    auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->iters = k;
        info->status = status;
        info->r0 = r0;
        info->relres = rel;
        info->t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        info->t_setup_ms = P.t_setup_ms;
        if (info->relres_history)
            for (int i = 0; i < std::min(k, info->history_cap); ++i)
                info->relres_history[i] = hs[kScalCount + kFlagCount / 2 + i];
    }
    if (status == IGA2L_ENUMERIC) throw Error{IGA2L_ENUMERIC, "residual diverged or became non-finite"};
    if (status == IGA2L_ENOTCONV) throw Error{IGA2L_ENOTCONV, "max_cycles reached before the tolerance"};
}

bool knots_open_uniform(const double *t, int nt, int p, int &m) {
    m = nt - 2 * p - 1;
    if (m < 2) return false;
    for (int i = 0; i < nt; ++i) {
        double expect = (i <= p) ? 0.0 : (i >= nt - p - 1 ? 1.0 : double(i - p) / m);
        if (!std::isfinite(t[i]) || std::fabs(t[i] - expect) > 1e-12) return false;
    }
    return true;
}

// nsweeps coloured FP64 sweeps on A u = b in place on u; w0, w1: two device
// vectors of n_fine doubles for the intermediate iterates (one kernel per
// colour, each reading the colour-start iterate and writing the next one:
// u -> w0 -> w1 -> w0 ... -> u)
void smooth_colour(const Problem &P, double *u, const double *b, int nsweeps, int S, double *w0, double *w1,
                   hipStream_t s) {
    const size_t bytes = sizeof(double) * size_t(P.fine.n);
    const int ncol = (P.dim == 3) ? S * S * S : S * S;
    double *w[2] = {w0, w1};
    for (int k = 0; k < nsweeps; ++k) {
        if (ncol == 1) {
            IGA2L_HIP(hipMemcpyAsync(w0, u, bytes, hipMemcpyDeviceToDevice, s));
            launch_colour_step<double>(P, 0, 0, 0, S, w0, u, b, false, s);
            continue;
        }
        const double *src = u;
        int c = 0;
        for (int cz = 0; cz < ((P.dim == 3) ? S : 1); ++cz)
            for (int cy = 0; cy < S; ++cy)
                for (int cx = 0; cx < S; ++cx, ++c) {
                    double *dst = (c == ncol - 1) ? u : w[c & 1];
                    launch_colour_step<double>(P, cx, cy, cz, S, src, dst, b, false, s);
                    src = dst;
                }
    }
}

// Fixed device array of iga2l_smooth_noalloc: its two intermediate iterates of
// at most IGA2L_NOALLOC_MAX_FINE doubles each.  Every device the library runs
// on holds its own copy until the process ends.  Host code never uses the
// array's name (a host-side stand-in); it uses the device address obtained
// once per device by scratch_on().
constexpr int64_t kNoAllocMaxFine = IGA2L_NOALLOC_MAX_FINE;
static __device__ __align__(256) double scratch[2 * kNoAllocMaxFine];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// device address of this device's copy of scratch; the caller has made the
// device current
double *scratch_on(int device) {
    IGA2L_REQUIRE(device >= 0 && device < kMaxDevices, IGA2L_EUNSUPPORTED, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        IGA2L_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        IGA2L_REQUIRE(ptr != nullptr, IGA2L_EDEVICE, "hipGetSymbolAddress returned no address");
        g_scratch_ptr[device] = static_cast<double *>(ptr);
    }
    return g_scratch_ptr[device];
}

}  // namespace
}  // namespace iga2l

using namespace iga2l;

extern "C" {

void iga2l_default_opts(iga2l_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-10;
    o->max_cycles = 100;
    o->ordering = IGA2L_COLOUR;
    o->colour_period = 0;
    o->coarse = IGA2L_COARSE_VCYCLE;
    o->nu1 = 1;
    o->nu2 = 1;
    o->precision = IGA2L_FP64;
    o->fine_post_sweeps = 0;
    o->lumped = 1;
    o->aggressive = 0;
    o->plow = 1;
}

const char *iga2l_last_error(void) { return g_last_error.c_str(); }

int iga2l_assemble(int dim, const double *const *knots, const int *nknots, int p, const double *kappa, int device,
                   iga2l_problem **out) {
    return guarded([&] {
        IGA2L_REQUIRE(out, IGA2L_EINVAL, "out is NULL");
        *out = nullptr;
        IGA2L_REQUIRE(dim == 2 || dim == 3, IGA2L_EINVAL, "dim must be 2 or 3");
        IGA2L_REQUIRE(p >= 1 && p <= kMaxP, IGA2L_EINVAL, "p must be in 1..8");
        IGA2L_REQUIRE(dim == 2 || p <= 4, IGA2L_EUNSUPPORTED, "3-D problems support p <= 4");
        IGA2L_REQUIRE(knots && nknots, IGA2L_EINVAL, "knots is NULL");
        int m = 0;
        for (int k = 0; k < dim; ++k) {
            IGA2L_REQUIRE(knots[k], IGA2L_EINVAL, "knot vector is NULL");
            IGA2L_REQUIRE(nknots[k] == nknots[0], IGA2L_EUNSUPPORTED, "all directions must use the same knots");
            int mk = 0;
            IGA2L_REQUIRE(knots_open_uniform(knots[k], nknots[k], p, mk), IGA2L_EINVAL,
                          "knots must be the open uniform vector (p+1 zeros, i/m, p+1 ones) with m >= 2");
            m = mk;
        }
        const auto t_start = std::chrono::steady_clock::now();
        auto *h = new iga2l_problem();
        try {
            Problem &P = h->P;
            P.device = device;
            P.dim = dim;
            P.p = p;
            P.m = m;
            int64_t ne = 1;
            for (int k = 0; k < dim; ++k) ne *= m;
            if (kappa) {
                P.kappa_one = false;
                P.kappa.assign(kappa, kappa + ne);
                for (double v : P.kappa)
                    IGA2L_REQUIRE(std::isfinite(v) && v > 0.0, IGA2L_EINVAL, "kappa must be finite and > 0");
            }
            set_device(P);
            host_assemble(P);
            P.layout_id = next_layout_id();
            IGA2L_HIP(hipDeviceSynchronize());
            P.t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

int iga2l_assemble_annulus(int p, int m, double r_in, double r_out, int device, iga2l_problem **out) {
    return guarded([&] {
        IGA2L_REQUIRE(out, IGA2L_EINVAL, "out is NULL");
        *out = nullptr;
        IGA2L_REQUIRE(p >= 2 && p <= kMaxP, IGA2L_EUNSUPPORTED, "annulus degree must be 2..8");
        IGA2L_REQUIRE(m >= 2, IGA2L_EINVAL, "need at least 2 elements per direction");
        IGA2L_REQUIRE(std::isfinite(r_in) && std::isfinite(r_out) && r_in > 0.0 && r_out > r_in, IGA2L_EINVAL,
                      "radii must satisfy 0 < r_in < r_out");
        const auto t_start = std::chrono::steady_clock::now();
        auto *h = new iga2l_problem();
        try {
            Problem &P = h->P;
            P.device = device;
            P.dim = 2;
            P.p = p;
            P.m = m;
            P.geometry = kGeomAnnulus;
            P.r_in = r_in;
            P.r_out = r_out;
            P.kappa_one = false;   // no interior stencil: the annulus rows all differ
            P.kappa.assign(size_t(m) * m, 1.0);
            set_device(P);
            host_assemble(P);
            P.layout_id = next_layout_id();
            IGA2L_HIP(hipDeviceSynchronize());
            P.t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

int iga2l_setup_blocks(iga2l_problem *prob, int block_width, const iga2l_opts *opts) {
    return guarded([&] {
        IGA2L_REQUIRE(prob, IGA2L_EINVAL, "problem is NULL");
        Problem &P = prob->P;
        set_device(P);
        iga2l_opts o = effective_opts(opts);
        int bw = block_width;
        if (bw == 0) bw = (P.p <= 4) ? 3 : (P.p <= 6 ? 5 : 7);
        IGA2L_REQUIRE(bw >= 1 && bw <= 7 && (bw & 1), IGA2L_EINVAL, "block width must be odd, 1..7");
        IGA2L_REQUIRE(P.dim == 2 || bw <= 3, IGA2L_EUNSUPPORTED, "3-D block width must be 1 or 3");
        hipStream_t s = nullptr;
        const auto t_start = std::chrono::steady_clock::now();
        auto tprev = t_start;
        auto stage = [&](const char *what) {   // IGA2L_TUNE_LOG=1: set-up stage times
            if (!tune_log()) return;
            IGA2L_HIP(hipDeviceSynchronize());
            const auto now = std::chrono::steady_clock::now();
            std::fprintf(stderr, "[iga2l setup] %s %.2f ms\n", what,
                         std::chrono::duration<double, std::milli>(now - tprev).count());
            tprev = now;
        };
        if (!P.blocks_ready || P.bw != bw) {
            P.blocks_ready = false;
            P.fp32_ready = false;
            P.tuned[0] = P.tuned[1] = false;
            P.bw = bw;
            P.bd = 1;
            for (int k = 0; k < P.dim; ++k) P.bd *= bw;
            std::vector<int> cls1;
            std::vector<int64_t> reps;
            host_block_classes(P, cls1, reps);
            P.cls_d.alloc(cls1.size() * sizeof(int));
            IGA2L_HIP(hipMemcpy(P.cls_d.ptr, cls1.data(), cls1.size() * sizeof(int), hipMemcpyHostToDevice));
            P.Inv64.alloc(size_t(P.nslots) * P.bd * P.bd * sizeof(double));
            stage("block classes");
            launch_block_inverse(P, reps, s);
            P.lex_off.clear();   // the lexicographic schedule is built on first use
            P.blocks_ready = true;
            stage("block inverses");
        }
        check_opts(P, o);
        if (o.plow != P.plow) {
            host_set_coarse_degree(P, o.plow);
            stage("coarse space");
        }
        if (o.precision == IGA2L_MIXED_FP32 && !P.fp32_ready) {
            P.A.v32.alloc(size_t(P.A.Wh) * P.A.npad * sizeof(float));
            launch_convert(P.A.v64.ptr, P.A.v32.ptr, int64_t(P.A.Wh) * P.A.npad, true, s);
            P.Inv32.alloc(size_t(P.nslots) * P.bd * P.bd * sizeof(float));
            launch_convert(P.Inv64.ptr, P.Inv32.ptr, P.nslots * P.bd * P.bd, true, s);
            P.R1d32.alloc(P.R1.size() * sizeof(float));
            launch_convert(P.R1d64.ptr, P.R1d32.ptr, int64_t(P.R1.size()), true, s);
            if (P.geometry == kGeomAnnulus) {
                P.R1yd32.alloc(P.R1y.size() * sizeof(float));
                launch_convert(P.R1yd64.ptr, P.R1yd32.ptr, int64_t(P.R1y.size()), true, s);
                const int64_t nf = 4 * int64_t(P.fine.n1) * (2 * P.p + 1);
                P.fac2d32.alloc(size_t(nf) * sizeof(float));
                launch_convert(P.fac2d64.ptr, P.fac2d32.ptr, nf, true, s);
            }
            P.dc64.alloc(size_t(P.coarse.n) * sizeof(double));
            P.ec64.alloc(size_t(P.coarse.n) * sizeof(double));
            IGA2L_HIP(hipStreamSynchronize(s));
            P.fp32_ready = true;
            stage("FP32 copies");
        }
        if ((o.coarse == IGA2L_COARSE_VCYCLE || o.aggressive) && !P.vcycle_ready) {
            host_build_levels(P);
            stage("V-cycle levels");
        }
        if (o.aggressive) {
            IGA2L_REQUIRE(P.levels.size() >= 2, IGA2L_EUNSUPPORTED,
                          "aggressive coarsening needs a V-cycle hierarchy with a 2h level (more than 512 coarse "
                          "unknowns)");
            if (o.coarse == IGA2L_COARSE_DIRECT && !P.agg_direct_ready) host_build_agg_direct(P);
        } else if (o.coarse == IGA2L_COARSE_DIRECT && !P.direct_ready) {
            IGA2L_REQUIRE(P.kappa_one || P.geometry == kGeomAnnulus || P.plow == 1, IGA2L_EUNSUPPORTED,
                          "the exact coarse solve with variable kappa needs the degree-1 coarse space");
            host_build_dst(P);
        }
        if (!o.lumped && !P.mass_ready) {
            host_build_mass(P);
            stage("exact transfers");
        }
        P.lumped_default = o.lumped != 0;
        IGA2L_HIP(hipDeviceSynchronize());
        // tile shapes of the coloured sweep, timed once per working precision
        // (not where every colour of the sweep runs the streamed kernel)
        const int S = o.colour_period ? o.colour_period : P.bw;
        const bool streamed = colour2d_stream_ok(P, S);
        if (P.dim == 2 && !P.tuned[0] && !streamed) {
            autotune_colour_tile<double>(P, S, s);
            P.tuned[0] = true;
        }
        if (P.dim == 2 && P.fp32_ready && !P.tuned[1] && !streamed) {
            autotune_colour_tile<float>(P, S, s);
            P.tuned[1] = true;
        }
        stage("tile autotuning");
        P.layout_id = next_layout_id();
        IGA2L_HIP(hipDeviceSynchronize());
        P.t_setup_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    });
}

int iga2l_sizes(const iga2l_problem *prob, int64_t *n_fine, int64_t *n_coarse, int64_t *n_elem) {
    return guarded([&] {
        IGA2L_REQUIRE(prob, IGA2L_EINVAL, "problem is NULL");
        if (n_fine) *n_fine = prob->P.fine.n;
        if (n_coarse) *n_coarse = prob->P.coarse.n;
        if (n_elem) *n_elem = prob->P.ne;
    });
}

int iga2l_residual(const iga2l_problem *prob, const double *u, const double *b, double *r, void *stream) {
    return guarded([&] {
        IGA2L_REQUIRE(prob && u && b && r, IGA2L_EINVAL, "null argument");
        IGA2L_REQUIRE(r != u, IGA2L_EINVAL, "r may not alias u");
        set_device(prob->P);
        launch_residual64(prob->P, u, b, r, false, false, false, static_cast<hipStream_t>(stream));
        IGA2L_HIP(hipGetLastError());
    });
}

int iga2l_smooth(const iga2l_problem *prob, double *u, const double *b, int nsweeps, const iga2l_opts *opts,
                 void *stream) {
    return guarded([&] {
        IGA2L_REQUIRE(prob && u && b, IGA2L_EINVAL, "null argument");
        IGA2L_REQUIRE(nsweeps >= 0, IGA2L_EINVAL, "nsweeps must be >= 0");
        Problem &P = const_cast<Problem &>(prob->P);
        IGA2L_REQUIRE(P.blocks_ready, IGA2L_EINVAL, "iga2l_setup_blocks must run first");
        iga2l_opts o = effective_opts(opts);
        o.precision = IGA2L_FP64;
        check_opts(P, o);
        set_device(P);
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (o.ordering == IGA2L_LEX) {
            if (P.lex_off.empty()) host_lex_schedule(P);
            for (int k = 0; k < nsweeps; ++k) {
                if (lex_sweep_fits(P)) launch_lex_sweep(P, u, b, s);
                else
                    for (size_t st = 0; st + 1 < P.lex_off.size(); ++st) launch_lex_step(P, int(st), u, b, s);
            }
        } else {
            const int S = o.colour_period ? o.colour_period : P.bw;
            smooth_colour(P, u, b, nsweeps, S, P.ework[0].as<double>(), P.ework[1].as<double>(), s);
        }
        IGA2L_HIP(hipGetLastError());
    });
}

int iga2l_smooth_noalloc(const iga2l_problem *prob, double *u, const double *b, int nsweeps,
                         const iga2l_opts *opts, void *stream) {
    return guarded([&] {
        IGA2L_REQUIRE(prob && u && b, IGA2L_EINVAL, "null argument");
        IGA2L_REQUIRE(nsweeps >= 0, IGA2L_EINVAL, "nsweeps must be >= 0");
        const Problem &P = prob->P;
        IGA2L_REQUIRE(P.fine.n <= kNoAllocMaxFine, IGA2L_EINVAL,
                      "iga2l_smooth_noalloc: n_fine = " + std::to_string(P.fine.n) +
                          " exceeds IGA2L_NOALLOC_MAX_FINE = " + std::to_string(kNoAllocMaxFine));
        IGA2L_REQUIRE(P.blocks_ready, IGA2L_EINVAL, "iga2l_setup_blocks must run first");
        iga2l_opts o = effective_opts(opts);
        o.precision = IGA2L_FP64;
        check_opts(P, o);
        IGA2L_REQUIRE(o.ordering == IGA2L_COLOUR, IGA2L_EUNSUPPORTED,
                      "iga2l_smooth_noalloc runs the coloured ordering only");
        set_device(P);
        double *w = scratch_on(P.device);
        const int S = o.colour_period ? o.colour_period : P.bw;
        smooth_colour(P, u, b, nsweeps, S, w, w + kNoAllocMaxFine, static_cast<hipStream_t>(stream));
        IGA2L_HIP(hipGetLastError());
    });
}

int iga2l_time_colour(const iga2l_problem *prob, int precision, int nsweeps, const iga2l_opts *opts, void *stream,
                      double *ms_per_launch) {
    return guarded([&] {
        IGA2L_REQUIRE(prob && ms_per_launch, IGA2L_EINVAL, "null argument");
        IGA2L_REQUIRE(nsweeps >= 1, IGA2L_EINVAL, "nsweeps must be >= 1");
        Problem &P = const_cast<Problem &>(prob->P);
        IGA2L_REQUIRE(P.blocks_ready, IGA2L_EINVAL, "iga2l_setup_blocks must run first");
        IGA2L_REQUIRE(precision == IGA2L_FP64 || (precision == IGA2L_MIXED_FP32 && P.fp32_ready), IGA2L_EINVAL,
                      "precision not set up");
        iga2l_opts o = effective_opts(opts);
        o.ordering = IGA2L_COLOUR;
        check_opts(P, o);
        set_device(P);
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int S = o.colour_period ? o.colour_period : P.bw;
        const int ncol = (P.dim == 3) ? S * S * S : S * S;
        const bool fp32 = precision == IGA2L_MIXED_FP32;
        // zero iterate and right-hand side (the arithmetic does not depend on the values)
        launch_fill_zero(P.ework[0].ptr, P.fine.n, fp32, s, nullptr);
        launch_fill_zero(P.ework[1].ptr, P.fine.n, fp32, s, nullptr);
        launch_fill_zero(P.rhs_w.ptr, P.fine.n, fp32, s, nullptr);
        auto sweep = [&]() {
            int cur = 0;
            for (int cz = 0; cz < ((P.dim == 3) ? S : 1); ++cz)
                for (int cy = 0; cy < S; ++cy)
                    for (int cx = 0; cx < S; ++cx) {
                        if (fp32)
                            launch_colour_step<float>(P, cx, cy, cz, S, P.ework[cur].as<float>(),
                                                      P.ework[1 - cur].as<float>(), P.rhs_w.as<float>(), false, s);
                        else
                            launch_colour_step<double>(P, cx, cy, cz, S, P.ework[cur].as<double>(),
                                                       P.ework[1 - cur].as<double>(), P.rhs_w.as<double>(), false, s);
                        cur = 1 - cur;
                    }
        };
        sweep();   // warm-up
        hipEvent_t e0, e1;
        IGA2L_HIP(hipEventCreate(&e0));
        IGA2L_HIP(hipEventCreate(&e1));
        float ms = 0.0f;
        hipError_t err = hipEventRecord(e0, s);
        for (int k = 0; k < nsweeps && err == hipSuccess; ++k) sweep();
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        IGA2L_HIP(err);
        *ms_per_launch = double(ms) / (double(nsweeps) * ncol);
    });
}

int iga2l_restrict(const iga2l_problem *prob, const double *r_fine, double *d_coarse, void *stream) {
    return guarded([&] {
        IGA2L_REQUIRE(prob && r_fine && d_coarse, IGA2L_EINVAL, "null argument");
        Problem &P = const_cast<Problem &>(prob->P);
        set_device(P);
        hipStream_t s = static_cast<hipStream_t>(stream);
        TransferGuard tg(P, !P.lumped_default);
        launch_restrict<double>(P, r_fine, d_coarse, s);
        if (P.transfer_exact) launch_mass_solve<double>(P, d_coarse, s);
        IGA2L_HIP(hipGetLastError());
    });
}

int iga2l_prolong(const iga2l_problem *prob, const double *e_coarse, double *u_fine, void *stream) {
    return guarded([&] {
        IGA2L_REQUIRE(prob && e_coarse && u_fine, IGA2L_EINVAL, "null argument");
        Problem &P = const_cast<Problem &>(prob->P);
        set_device(P);
        hipStream_t s = static_cast<hipStream_t>(stream);
        TransferGuard tg(P, !P.lumped_default);
        const double *ec = e_coarse;
        if (P.transfer_exact) {
            IGA2L_HIP(hipMemcpyAsync(P.ec.ptr, e_coarse, sizeof(double) * size_t(P.coarse.n), hipMemcpyDeviceToDevice, s));
            launch_mass_solve<double>(P, P.ec.as<double>(), s);
            ec = P.ec.as<double>();
        }
        launch_prolong_add<double>(P, ec, u_fine, s);
        IGA2L_HIP(hipGetLastError());
    });
}

int iga2l_coarse_solve(const iga2l_problem *prob, const double *d_coarse, double *e_coarse, const iga2l_opts *opts,
                       void *stream) {
    return guarded([&] {
        IGA2L_REQUIRE(prob && d_coarse && e_coarse, IGA2L_EINVAL, "null argument");
        IGA2L_REQUIRE(d_coarse != e_coarse, IGA2L_EINVAL, "e_coarse may not alias d_coarse");
        Problem &P = const_cast<Problem &>(prob->P);
        iga2l_opts o = effective_opts(opts);
        check_opts(P, o);
        set_device(P);
        coarse_solve<double>(P, o, d_coarse, e_coarse, static_cast<hipStream_t>(stream));
        IGA2L_HIP(hipGetLastError());
    });
}

int iga2l_solve(const iga2l_problem *prob, const double *b, double *u, const iga2l_opts *opts, iga2l_info *info,
                void *stream) {
    return guarded([&] {
        IGA2L_REQUIRE(prob, IGA2L_EINVAL, "problem is NULL");
        Problem &P = const_cast<Problem &>(prob->P);
        iga2l_opts o = effective_opts(opts);
        check_opts(P, o);
        set_device(P);
        solve_impl(P, b, u, o, info, static_cast<hipStream_t>(stream));
    });
}

int iga2l_solve_batch(iga2l_problem *const *probs, int nprob, const double *const *b, double *const *u,
                      const iga2l_opts *opts, iga2l_info *infos, void *stream) {
    return guarded([&] {
        IGA2L_REQUIRE(nprob >= 0 && (nprob == 0 || (probs && b && u)), IGA2L_EINVAL, "null argument");
        iga2l_opts o = effective_opts(opts);
        int worst = IGA2L_OK;
        std::string msg;
        std::vector<Problem *> pv(size_t(std::max(nprob, 0)));
        for (int k = 0; k < nprob; ++k) {
            IGA2L_REQUIRE(probs[k], IGA2L_EINVAL, "problem is NULL");
            pv[k] = &probs[k]->P;
            check_opts(*pv[k], o);
        }
        if (batch_supported(pv.data(), nprob, o)) {
            set_device(*pv[0]);
            solve_batch_fused(pv.data(), nprob, b, u, o, infos, static_cast<hipStream_t>(stream), worst, msg);
            if (worst != IGA2L_OK) throw Error{worst, msg};
            return;
        }
        for (int k = 0; k < nprob; ++k) {
            Problem &P = *pv[k];
            set_device(P);
            try {
                solve_impl(P, b[k], u[k], o, infos ? &infos[k] : nullptr, static_cast<hipStream_t>(stream));
            } catch (const Error &e) {
                if (e.code == IGA2L_ENOTCONV || e.code == IGA2L_ENUMERIC) {
                    if (worst == IGA2L_OK || e.code == IGA2L_ENUMERIC) {
                        worst = e.code;
                        msg = "problem " + std::to_string(k) + ": " + e.msg;
                    }
                } else {
                    throw;
                }
            }
        }
        if (worst != IGA2L_OK) throw Error{worst, msg};
    });
}

int iga2l_solve_backward(const iga2l_problem *prob, const double *u, const double *grad_u, double *lambda,
                         double *grad_kappa, const iga2l_opts *opts, iga2l_info *info, void *stream) {
    return guarded([&] {
        IGA2L_REQUIRE(prob && u && grad_u && lambda, IGA2L_EINVAL, "null argument");
        Problem &P = const_cast<Problem &>(prob->P);
        IGA2L_REQUIRE(!grad_kappa || P.geometry == kGeomSquare, IGA2L_EUNSUPPORTED,
                      "the coefficient gradient is defined on the square (the annulus has no kappa)");
        iga2l_opts o = effective_opts(opts);
        check_opts(P, o);
        set_device(P);
        hipStream_t s = static_cast<hipStream_t>(stream);
        IGA2L_HIP(hipMemsetAsync(lambda, 0, sizeof(double) * size_t(P.fine.n), s));
        // A is symmetric: the adjoint system A lambda = dL/du uses the same solver
        solve_impl(P, grad_u, lambda, o, info, s);
        if (grad_kappa) {
            launch_grad_kappa(P, u, lambda, grad_kappa, s);
            IGA2L_HIP(hipGetLastError());
            IGA2L_HIP(hipStreamSynchronize(s));
        }
    });
}

void iga2l_destroy(iga2l_problem *prob) {
    if (!prob) return;
    (void)hipSetDevice(prob->P.device);
    (void)hipDeviceSynchronize();
    delete prob;
}

}  // extern "C"
