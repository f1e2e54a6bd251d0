// batch.hip -- solve of many independent 2-D problems with batched launches.
//
// Every step of the correction cycle (each colour of the Schwarz sweep, the
// defect, the restriction, each level of the V-cycle, the prolongation and
// update, the FP64 residual with its norm and convergence test) is one launch
// per kernel variant for the whole batch instead of one per problem.  A
// workgroup finds its problem and tile in a precomputed map and reads that
// problem's operands from a device table; problems that have converged stop
// at once through their own flag.  The arithmetic of every tile equals that of
// the single-problem kernels, so the results equal those of separate solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "internal.h"

namespace iga2l {

uint64_t next_layout_id() {
    static std::atomic<uint64_t> counter{0};
    return ++counter;
}

namespace {

inline int cdiv(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// copies each problem's status block (scalars, flags, history) into one array
__global__ void kb_gather_status(const BatchProb *__restrict__ bp, double *__restrict__ out, int stride, int nwords) {
    const double *src = bp[blockIdx.x].scal;
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) out[int64_t(blockIdx.x) * stride + i] = src[i];
}

struct Group {
    int p = 0, bw = 0, S = 0, nbx = 0, nby = 0;
    DevBuf res_map, col_map;
    int res_nwg = 0, col_nwg = 0;
};

struct Plan {
    int device = 0;
    std::vector<uint64_t> ids;
    int precision = 0, colour_period = 0, nu1 = 0, nu2 = 0;
    int nprob = 0;
    BatchProb *host_table = nullptr;   // pinned
    DevBuf table;                      // BatchProb[nprob]
    std::vector<Group> groups;
    DevBuf tr_map, pr_map;
    int tr_nwg = 0, pr_nwg = 0;
    size_t tr_shm = 0, pr_shm = 0;
    std::vector<DevBuf> lev_args, lev_maps;   // per depth of the multi-workgroup V-cycle levels
    std::vector<int> lev_nwg;
    DevBuf bottom_args;
    size_t bottom_shm = 0;
    int hist_cap = 0;
    int status_stride = 0;             // doubles per problem in the gathered status
    DevBuf status_dev;
    double *status_host = nullptr;     // pinned
    int expected_cycles = 1;
    // one cycle (correction cycle + FP64 residual, norm and convergence test)
    // captured into a HIP graph, replayed once per cycle
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;

    ~Plan() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (host_table) (void)hipHostFree(host_table);
        if (status_host) (void)hipHostFree(status_host);
    }
};

std::mutex g_plan_mutex;
Plan *g_plan = nullptr;   // the last plan; replaced when the batch changes

DevBuf upload_map(const std::vector<int2> &m) {
    DevBuf d;
    d.alloc(std::max<size_t>(1, m.size()) * sizeof(int2));
    if (!m.empty()) IGA2L_HIP(hipMemcpy(d.ptr, m.data(), m.size() * sizeof(int2), hipMemcpyHostToDevice));
    return d;
}

template <class T>
size_t bottom_of(const Problem &P) { return std::is_same<T, double>::value ? P.vc_bottom64 : P.vc_bottom32; }

template <class T>
const LevelDev<T> &levhost_of(const Problem &P, size_t l) {
    if constexpr (std::is_same<T, double>::value) return P.levhost64[l];
    else return P.levhost32[l];
}

template <class T>
const LevelDev<T> *levdev_of(const Problem &P) {
    return std::is_same<T, double>::value ? reinterpret_cast<const LevelDev<T> *>(P.levdev64.ptr)
                                          : reinterpret_cast<const LevelDev<T> *>(P.levdev32.ptr);
}

template <class T>
void build_vcycle(Plan &pl, const std::vector<Problem *> &probs) {
    size_t depth = 0;
    for (Problem *P : probs) depth = std::max(depth, bottom_of<T>(*P));
    pl.lev_args.clear();
    pl.lev_maps.clear();
    pl.lev_nwg.clear();
    for (size_t d = 0; d < depth; ++d) {
        std::vector<BatchLevel<T>> args;
        std::vector<int2> map;
        for (Problem *P : probs) {
            if (bottom_of<T>(*P) <= d) continue;
            const Level &L = P->levels[d];
            const Level &C = P->levels[d + 1];
            BatchLevel<T> a{};
            a.L = levhost_of<T>(*P, d);
            a.rhs = (d == 0) ? P->dc.as<T>() : L.rhs.as<T>();
            a.e_pre = L.e[0].as<T>();
            a.rc = C.rhs.as<T>();
            a.ecl = C.res.as<T>();
            a.e_out = (d == 0) ? P->ec.as<T>() : L.res.as<T>();
            a.n1c = C.g.n1;
            a.ntx = cdiv(L.g.n1, 32);
            a.nty = cdiv(L.g.n1, 8);
            a.skip = dev_flags(*P);
            const int k = int(args.size());
            for (int t = 0; t < a.ntx * a.nty; ++t) map.push_back(make_int2(k, t));
            args.push_back(a);
        }
        DevBuf da;
        da.alloc(args.size() * sizeof(BatchLevel<T>));
        IGA2L_HIP(hipMemcpy(da.ptr, args.data(), args.size() * sizeof(BatchLevel<T>), hipMemcpyHostToDevice));
        pl.lev_args.push_back(std::move(da));
        pl.lev_maps.push_back(upload_map(map));
        pl.lev_nwg.push_back(int(map.size()));
    }
    std::vector<BatchBottom<T>> bb;
    pl.bottom_shm = 0;
    for (Problem *P : probs) {
        const size_t lb = bottom_of<T>(*P);
        BatchBottom<T> a{};
        a.levels = levdev_of<T>(*P) + lb;
        a.nlev = int(P->levels.size() - lb);
        a.rhs = (lb == 0) ? P->dc.as<T>() : P->levels[lb].rhs.as<T>();
        a.e = (lb == 0) ? P->ec.as<T>() : P->levels[lb].res.as<T>();
        a.skip = dev_flags(*P);
        bb.push_back(a);
        pl.bottom_shm = std::max(pl.bottom_shm, size_t(vcycle_bottom_lds(*P, lb)) * sizeof(T));
    }
    pl.bottom_args.alloc(bb.size() * sizeof(BatchBottom<T>));
    IGA2L_HIP(hipMemcpy(pl.bottom_args.ptr, bb.data(), bb.size() * sizeof(BatchBottom<T>), hipMemcpyHostToDevice));
}

// colour tiles of a group for the shape (nbx, nby): per-problem tile grids
// covering every colour, and the workgroup map
void colour_layout(Plan &pl, Group &g, const std::vector<int> &members) {
    std::vector<int2> cm;
    for (int k : members) {
        BatchProb &q = pl.host_table[k];
        q.col_ntx = cdiv(q.n1 + g.S - 1, g.nbx * g.S);
        q.col_nty = cdiv(q.n1 + g.S - 1, g.nby * g.S);
        for (int t = 0; t < q.col_ntx * q.col_nty; ++t) cm.push_back(make_int2(k, t));
    }
    g.col_map = upload_map(cm);
    g.col_nwg = int(cm.size());
}

// Autotuner of the batched coloured sweep: every candidate tile shape runs
// one colour of the whole group on its own workspaces (numerics-neutral: a
// point's arithmetic does not depend on the tile); the fastest is kept.
void tune_group(Plan &pl, Group &g, const std::vector<int> &members, bool fp32) {
    int n1max = 0;
    for (int k : members) n1max = std::max(n1max, pl.host_table[k].n1);
    auto cands = colour_tile_candidates(g.S, n1max);
    hipEvent_t e0, e1;
    IGA2L_HIP(hipEventCreate(&e0));
    IGA2L_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int bx = 4, by = 4;
    colour_tile_clamp(g.S, bx, by);
    const int rhs_role = fp32 ? kVecRhsW : kVecR64;
    const BatchProb *tb = pl.table.as<BatchProb>();
    auto launch = [&]() {
        if (fp32)
            launch_colour_batch<float>(tb, g.col_map.as<int2>(), g.col_nwg, g.p, g.bw, g.nbx, g.nby, 1 % g.S, 1 % g.S,
                                       g.S, kVecE0, kVecE1, rhs_role, false, false, nullptr, false);
        else
            launch_colour_batch<double>(tb, g.col_map.as<int2>(), g.col_nwg, g.p, g.bw, g.nbx, g.nby, 1 % g.S,
                                        1 % g.S, g.S, kVecE0, kVecE1, rhs_role, false, false, nullptr, false);
    };
    try {
        for (auto [cbx, cby] : cands) {
            g.nbx = cbx;
            g.nby = cby;
            colour_layout(pl, g, members);
            IGA2L_HIP(hipMemcpy(pl.table.ptr, pl.host_table, pl.nprob * sizeof(BatchProb), hipMemcpyHostToDevice));
            launch();
            IGA2L_HIP(hipEventRecord(e0, nullptr));
            for (int r = 0; r < 3; ++r) launch();
            IGA2L_HIP(hipEventRecord(e1, nullptr));
            IGA2L_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            IGA2L_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (tune_log())
                std::fprintf(stderr, "[iga2l tune] batch p=%d b=%d s=%d %d problems: tile %dx%d blocks %.2f us\n", g.p,
                             g.bw, g.S, int(members.size()), cbx, cby, 1e3f * ms / 3);
            if (ms < best) {
                best = ms;
                bx = cbx;
                by = cby;
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g.nbx = bx;
    g.nby = by;
    colour_layout(pl, g, members);
}

std::unique_ptr<Plan> build_plan(const std::vector<Problem *> &probs, const iga2l_opts &o) {
    auto pl = std::make_unique<Plan>();
    const int n = int(probs.size());
    pl->device = probs[0]->device;
    pl->nprob = n;
    pl->precision = o.precision;
    pl->colour_period = o.colour_period;
    pl->nu1 = o.nu1;
    pl->nu2 = o.nu2;
    for (Problem *P : probs) pl->ids.push_back(P->layout_id);
    const bool fp32 = o.precision == IGA2L_MIXED_FP32;
    const size_t elem = fp32 ? sizeof(float) : sizeof(double);

    IGA2L_HIP(hipHostMalloc(reinterpret_cast<void **>(&pl->host_table), n * sizeof(BatchProb), hipHostMallocDefault));
    pl->hist_cap = probs[0]->hist_cap;
    int expected = 1;
    std::map<std::tuple<int, int, int>, std::vector<int>> group_of;
    std::vector<int2> tr_map, pr_map;
    for (int k = 0; k < n; ++k) {
        const Problem &P = *probs[k];
        BatchProb q{};
        q.val[0] = P.A.v64.ptr;
        q.val[1] = P.A.v32.ptr;
        q.inv[0] = P.Inv64.ptr;
        q.inv[1] = P.Inv32.ptr;
        q.cs[0] = P.cs64.ptr;
        q.cs[1] = P.cs32.ptr;
        q.fac[0] = colour_factor_rows(P, true);
        q.fac[1] = colour_factor_rows(P, false);
        q.R1[0] = P.R1d64.ptr;
        q.R1[1] = P.R1d32.ptr;
        q.cls = P.cls_d.as<int>();
        q.clsL = class_split(P);
        q.npad = P.A.npad;
        q.pitch1 = P.A.pitch[1];
        q.n1 = P.fine.n1;
        q.n1c = P.coarse.n1;
        q.p = P.p;
        q.ncls1 = P.ncls1;
        q.ulo = P.ulo;
        q.uhi = P.uhi;
        q.hist_cap = P.hist_cap;
        q.scal = P.scal.as<double>();
        q.partial = P.partial.as<double>();
        q.hist = dev_hist(P);
        q.flags = dev_flags(P);
        q.vec[kVecR64] = P.r64.ptr;
        q.vec[kVecE0] = P.ework[0].ptr;
        q.vec[kVecE1] = P.ework[1].ptr;
        q.vec[kVecRhsW] = P.rhs_w.ptr;
        q.vec[kVecDFine] = P.dfine.ptr;
        q.vec[kVecDC] = P.dc.ptr;
        q.vec[kVecEC] = P.ec.ptr;
        q.res_ntx = cdiv(q.n1, 64);
        q.res_nty = cdiv(q.n1, 4);
        IGA2L_REQUIRE(int64_t(q.res_ntx) * q.res_nty <= P.npartial, IGA2L_EUNSUPPORTED,
                      "grid too large for the norm workspace");
        transfer_tile_2d(q.n1c, q.tr_cx, q.tr_cy);
        q.tr_ntx = cdiv(q.n1c, q.tr_cx);
        q.tr_nty = cdiv(q.n1c, q.tr_cy);
        transfer_tile_2d(q.n1, q.pr_tx, q.pr_ty);
        q.pr_ntx = cdiv(q.n1, q.pr_tx);
        q.pr_nty = cdiv(q.n1, q.pr_ty);
        for (int t = 0; t < q.tr_ntx * q.tr_nty; ++t) tr_map.push_back(make_int2(k, t));
        for (int t = 0; t < q.pr_ntx * q.pr_nty; ++t) pr_map.push_back(make_int2(k, t));
        pl->tr_shm = std::max(pl->tr_shm, restrict2d_lds(P.p, q.tr_cx, q.tr_cy, elem));
        pl->pr_shm = std::max(pl->pr_shm, prolong2d_lds(P.p, q.pr_tx, q.pr_ty, elem));
        const int S = o.colour_period ? o.colour_period : P.bw;
        group_of[std::make_tuple(P.p, P.bw, S)].push_back(k);
        pl->host_table[k] = q;
        expected = std::max(expected, P.expected_cycles);
    }
    pl->expected_cycles = expected;
    pl->table.alloc(n * sizeof(BatchProb));
    for (auto &kv : group_of) {
        Group g;
        std::tie(g.p, g.bw, g.S) = kv.first;
        std::vector<int2> rm;
        for (int k : kv.second) {
            const BatchProb &q = pl->host_table[k];
            for (int t = 0; t < q.res_ntx * q.res_nty; ++t) rm.push_back(make_int2(k, t));
        }
        g.res_map = upload_map(rm);
        g.res_nwg = int(rm.size());
        tune_group(*pl, g, kv.second, fp32);
        pl->groups.push_back(std::move(g));
    }
    pl->tr_map = upload_map(tr_map);
    pl->tr_nwg = int(tr_map.size());
    pl->pr_map = upload_map(pr_map);
    pl->pr_nwg = int(pr_map.size());
    if (fp32) build_vcycle<float>(*pl, probs);
    else build_vcycle<double>(*pl, probs);
    pl->status_stride = kScalCount + kFlagCount / 2 + pl->hist_cap;
    pl->status_dev.alloc(size_t(n) * pl->status_stride * sizeof(double));
    IGA2L_HIP(hipHostMalloc(reinterpret_cast<void **>(&pl->status_host), size_t(n) * pl->status_stride * sizeof(double),
                            hipHostMallocDefault));
    return pl;
}

template <class T>
void batch_cycle(const Plan &pl, hipStream_t s) {
    const BatchProb *tb = pl.table.as<BatchProb>();
    const bool fp32 = !std::is_same<T, double>::value;
    const int rhs_role = fp32 ? kVecRhsW : kVecR64;
    int ncol_max = 0;
    for (const Group &g : pl.groups) ncol_max = std::max(ncol_max, g.S * g.S);
    // colour c of every group at step c (colours of different problems are independent)
    for (int c = 0; c < ncol_max; ++c)
        for (const Group &g : pl.groups) {
            if (c >= g.S * g.S) continue;
            const int src = kVecE0 + (c & 1), dst = kVecE0 + 1 - (c & 1);
            launch_colour_batch<T>(tb, g.col_map.as<int2>(), g.col_nwg, g.p, g.bw, g.nbx, g.nby, c % g.S, c / g.S,
                                   g.S, src, dst, rhs_role, c == 0, fp32 && c == 0, s);
        }
    int e_role = -1;
    for (const Group &g : pl.groups) {
        const int er = kVecE0 + ((g.S * g.S) & 1);
        IGA2L_REQUIRE(e_role < 0 || e_role == er, IGA2L_EUNSUPPORTED, "colour counts of different parity in one batch");
        e_role = er;
        launch_residual_batch_dispatch<T>(g.p, tb, g.res_map.as<int2>(), g.res_nwg, er, rhs_role, kVecDFine, false,
                                          true, s);
    }
    launch_restrict_batch<T>(tb, pl.tr_map.as<int2>(), pl.tr_nwg, pl.tr_shm, kVecDFine, kVecDC, s);
    const int depth = int(pl.lev_args.size());
    for (int d = 0; d < depth; ++d)
        launch_rb_multi2_batch<T>(pl.lev_args[d].as<BatchLevel<T>>(), pl.lev_maps[d].as<int2>(), pl.lev_nwg[d], pl.nu1,
                                  true, true, s);
    launch_vcycle_bottom_batch<T>(pl.bottom_args.as<BatchBottom<T>>(), pl.nprob, pl.bottom_shm, pl.nu1, pl.nu2, s);
    for (int d = depth - 1; d >= 0; --d)
        launch_rb_multi2_batch<T>(pl.lev_args[d].as<BatchLevel<T>>(), pl.lev_maps[d].as<int2>(), pl.lev_nwg[d], pl.nu2,
                                  false, pl.nu1 == 0, s);
    launch_prolong_update_batch<T>(tb, pl.pr_map.as<int2>(), pl.pr_nwg, pl.pr_shm, kVecEC, e_role, fp32, s);
}

// FP64 residual, norm and (book) the convergence test after a cycle; the
// residual before the first cycle ignores the stop flags (they still hold the
// previous solve's state until the initialisation)
void batch_residual(const Plan &pl, bool fp32, bool book, hipStream_t s) {
    const BatchProb *tb = pl.table.as<BatchProb>();
    for (const Group &g : pl.groups)
        launch_residual_batch_dispatch<double>(g.p, tb, g.res_map.as<int2>(), g.res_nwg, kVecU, kVecB, kVecR64, true,
                                               book, s);
    launch_norm_finalize_batch(tb, pl.nprob, fp32, book, s);
}

// IGA2L_BATCH_GRAPH=0 in the environment: launch the kernels of every cycle
// directly instead of replaying the captured graph (same kernels, same results)
bool batch_graph_enabled() {
    const char *e = std::getenv("IGA2L_BATCH_GRAPH");
    return !(e && e[0] == '0');
}

// Captures one cycle of the plan (kernel launches only: no memset or copy
// nodes) on a private stream of default priority and instantiates it.  The
// kernels read every problem's vectors through the device table, so the graph
// stays valid for every call with the same plan.
void ensure_graph(Plan &pl, bool fp32) {
    if (pl.gexec) return;
    if (!pl.cap_stream) IGA2L_HIP(hipStreamCreateWithFlags(&pl.cap_stream, hipStreamNonBlocking));
    IGA2L_HIP(hipStreamBeginCapture(pl.cap_stream, hipStreamCaptureModeThreadLocal));
    try {
        if (fp32) batch_cycle<float>(pl, pl.cap_stream);
        else batch_cycle<double>(pl, pl.cap_stream);
        batch_residual(pl, fp32, true, pl.cap_stream);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(pl.cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    IGA2L_HIP(hipStreamEndCapture(pl.cap_stream, &pl.graph));
    IGA2L_HIP(hipGraphInstantiate(&pl.gexec, pl.graph, nullptr, nullptr, 0));
}

}  // namespace

bool batch_supported(Problem *const *probs, int nprob, const iga2l_opts &o) {
    if (nprob < 2) return false;
    if (o.ordering != IGA2L_COLOUR || o.coarse != IGA2L_COARSE_VCYCLE || o.fine_post_sweeps != 0) return false;
    if (!o.lumped || o.aggressive || o.plow != 1) return false;   // other coarse spaces: problem by problem
    if (o.nu1 < 0 || o.nu1 > 4 || o.nu2 < 1 || o.nu2 > 4) return false;
    for (int k = 0; k < nprob; ++k) {
        const Problem &P = *probs[k];
        if (P.dim != 2 || P.fine.n >= (int64_t(1) << 20) || P.device != probs[0]->device) return false;
        if (!P.blocks_ready || !P.vcycle_ready) return false;
        if (o.precision == IGA2L_MIXED_FP32 && !P.fp32_ready) return false;
    }
    return true;
}

// Batched solve loop: the same device-side convergence book-keeping as the
// single-problem loop, with one status gather per synchronisation.
void solve_batch_fused(Problem *const *probs, int nprob, const double *const *b, double *const *u,
                       const iga2l_opts &o, iga2l_info *infos, hipStream_t s, int &worst, std::string &msg) {
    std::vector<Problem *> pv(probs, probs + nprob);
    const int cap = std::max(o.max_cycles, 1);
    for (Problem *P : pv) ensure_history(*P, cap);
    // all problems of a plan share one history capacity
    int hist_cap = 0;
    for (Problem *P : pv) hist_cap = std::max(hist_cap, P->hist_cap);
    for (Problem *P : pv) ensure_history(*P, hist_cap);

    std::lock_guard<std::mutex> lock(g_plan_mutex);
    bool reuse = g_plan && g_plan->nprob == nprob && g_plan->precision == o.precision &&
                 g_plan->colour_period == o.colour_period && g_plan->nu1 == o.nu1 && g_plan->nu2 == o.nu2 &&
                 g_plan->device == pv[0]->device && g_plan->hist_cap == hist_cap;
    for (int k = 0; reuse && k < nprob; ++k) reuse = g_plan->ids[k] == pv[k]->layout_id;
    if (!reuse) {
        delete g_plan;
        g_plan = nullptr;
        g_plan = build_plan(pv, o).release();
    }
    Plan &pl = *g_plan;
    for (int k = 0; k < nprob; ++k) {
        IGA2L_REQUIRE(b[k] && u[k], IGA2L_EINVAL, "null vector");
        pl.host_table[k].vec[kVecU] = u[k];
        pl.host_table[k].vec[kVecB] = const_cast<double *>(b[k]);
    }
    auto t0 = std::chrono::steady_clock::now();
    IGA2L_HIP(hipMemcpyAsync(pl.table.ptr, pl.host_table, nprob * sizeof(BatchProb), hipMemcpyHostToDevice, s));
    const bool fp32 = o.precision == IGA2L_MIXED_FP32;
    const BatchProb *tb = pl.table.as<BatchProb>();
    batch_residual(pl, fp32, false, s);
    launch_solve_init_batch(tb, nprob, o.tol, o.max_cycles, s);
    int issued = 0;
    int batch = std::max(1, std::min(pl.expected_cycles, o.max_cycles));
    const int fixed = kScalCount + kFlagCount / 2;
    const bool graph = batch_graph_enabled();
    if (graph) ensure_graph(pl, fp32);
    while (true) {
        for (int j = 0; j < batch && issued < o.max_cycles; ++j, ++issued) {
            if (graph) {
                IGA2L_HIP(hipGraphLaunch(pl.gexec, s));
            } else {
                if (fp32) batch_cycle<float>(pl, s);
                else batch_cycle<double>(pl, s);
                batch_residual(pl, fp32, true, s);
            }
        }
        IGA2L_HIP(hipGetLastError());
        const int words = fixed + std::min(issued, pl.hist_cap);
        hipLaunchKernelGGL(kb_gather_status, dim3(nprob), dim3(256), 0, s, tb, pl.status_dev.as<double>(),
                           pl.status_stride, words);
        IGA2L_HIP(hipMemcpyAsync(pl.status_host, pl.status_dev.ptr, size_t(nprob) * pl.status_stride * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
        IGA2L_HIP(hipStreamSynchronize(s));
        bool all_done = true;
        for (int k = 0; k < nprob; ++k) {
            const int *hf = reinterpret_cast<const int *>(pl.status_host + size_t(k) * pl.status_stride + kScalCount);
            all_done = all_done && hf[kFlagDone];
        }
        if (all_done || issued >= o.max_cycles) break;
        batch = 2;
    }
    auto t1 = std::chrono::steady_clock::now();
    int most = 0;
    for (int k = 0; k < nprob; ++k) {
        const double *hs = pl.status_host + size_t(k) * pl.status_stride;
        const int *hf = reinterpret_cast<const int *>(hs + kScalCount);
        const int it = hf[kFlagIter];
        const double r0 = hs[kScalR0];
        const double rel = (it > 0) ? hs[fixed + it - 1] : (r0 > 0 ? 1.0 : 0.0);
        int status = IGA2L_OK;
        if (hf[kFlagStatus] == 2) status = IGA2L_ENUMERIC;
        else if (hf[kFlagStatus] == 1 || (!hf[kFlagDone] && rel > o.tol)) status = IGA2L_ENOTCONV;
        if (it > 0) pv[k]->expected_cycles = it;
        most = std::max(most, it);
        if (infos) {
            iga2l_info &inf = infos[k];
            inf.iters = it;
            inf.status = status;
            inf.r0 = r0;
            inf.relres = rel;
            inf.t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
            inf.t_setup_ms = pv[k]->t_setup_ms;
            if (inf.relres_history)
                for (int i = 0; i < std::min(it, std::min(inf.history_cap, pl.hist_cap)); ++i)
                    inf.relres_history[i] = hs[fixed + i];
        }
        // report the first non-converged problem, or the first numerical failure
        if (status != IGA2L_OK && worst != IGA2L_ENUMERIC && (worst == IGA2L_OK || status == IGA2L_ENUMERIC)) {
            worst = status;
            msg = "problem " + std::to_string(k) + ": " +
                  (status == IGA2L_ENUMERIC ? "residual diverged or became non-finite"
                                            : "max_cycles reached before the tolerance");
        }
    }
    if (most > 0) pl.expected_cycles = most;
}

}  // namespace iga2l
