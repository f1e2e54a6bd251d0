// kernels_vcycle.hip -- the degree-1 h-multigrid V(nu1,nu2) cycle of the
// coarse level (red-black Gauss-Seidel, linear interpolation onto the
// odd-indexed nodes, Galerkin operators, exact solve of the first level with at
// most kCoarsestMax unknowns by its precomputed dense inverse).
//
// Fine levels of the hierarchy run one kernel per full red-black step (tiles
// with a halo of 2: the red half step is recomputed on the tile's halo ring so
// that the black half step needs no grid-wide barrier) and one tiled
// residual-restriction kernel; the prolongation is fused into the load of the
// first post-smoothing step.  All levels whose vectors fit in the LDS of one
// workgroup run inside a single-workgroup kernel.  A red (black) half step
// updates every red (black) point from the iterate at the start of the half
// step.  Levels whose operator is translation invariant (kappa = 1) use the
// interior stencil as constants instead of loading coefficients.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include "internal.h"

namespace iga2l {

namespace {

inline unsigned nblk(int64_t n, int t) { return unsigned((n + t - 1) / t); }

template <int D>
struct VT;  // tile shapes of the multi-workgroup kernels
template <>
struct VT<2> {
    static constexpr int TX = 32, TY = 8, TZ = 1;   // red-black step tile
    static constexpr int CX = 16, CY = 16, CZ = 1;  // residual-restriction coarse tile
};
template <>
struct VT<3> {
    static constexpr int TX = 16, TY = 8, TZ = 4;
    static constexpr int CX = 8, CY = 8, CZ = 4;
};

template <int D>
__device__ __forceinline__ int w_of(int ox, int oy, int oz) {
    return (D == 3) ? ((oz + 1) * 3 + (oy + 1)) * 3 + (ox + 1) : (oy + 1) * 3 + (ox + 1);
}

// Stencil coefficient A[i][i+o] of a level.
template <int D, class T>
__device__ __forceinline__ T coef(const LevelDev<T> &L, int64_t i, int w) {
    return L.cst ? L.c[w] : L.S[int64_t(w) * L.n + i];
}
template <int D, class T>
__device__ __forceinline__ T inv_diag(const LevelDev<T> &L, int64_t i) {
    return L.cst ? L.cinv : L.invd[i];
}

// parents of a fine index v in 1-D (coarse node I sits at fine index 2I+1)
template <class T>
__device__ __forceinline__ int parents(int v, int n1c, int *I, T *w) {
    int c = 0;
    if (v & 1) {
        I[c] = (v - 1) >> 1;
        w[c++] = T(1);
    } else {
        if ((v >> 1) - 1 >= 0) { I[c] = (v >> 1) - 1; w[c++] = T(0.5); }
        if ((v >> 1) < n1c) { I[c] = v >> 1; w[c++] = T(0.5); }
    }
    return c;
}

// (P ec)[i] for a fine index (ix,iy,iz), ec on the coarse grid n1c
template <int D, class T>
__device__ __forceinline__ T interp_value(const T *__restrict__ ec, int n1c, int ix, int iy, int iz) {
    int Ix[2], Iy[2], Iz[2];
    T wx[2], wy[2], wz[2];
    const int nx = parents<T>(ix, n1c, Ix, wx), ny = parents<T>(iy, n1c, Iy, wy);
    int nz = 1;
    Iz[0] = 0;
    wz[0] = T(1);
    if (D == 3) nz = parents<T>(iz, n1c, Iz, wz);
    T acc = T(0);
    for (int c = 0; c < nz; ++c)
        for (int b = 0; b < ny; ++b)
            for (int a = 0; a < nx; ++a)
                acc += wz[c] * wy[b] * wx[a] * ec[(int64_t(Iz[c]) * n1c + Iy[b]) * n1c + Ix[a]];
    return acc;
}

// --------------------------------------------------------------------------
// One full red-black step on a level:  e_dst = S_black S_red (e_in)  with
// e_in = (zero_src ? 0 : e_src) + (ec ? P ec : 0).
template <int D, class T>
__global__ void __launch_bounds__(256) k_rb_step(LevelDev<T> L, const T *__restrict__ e_src, int zero_src,
                                                 const T *__restrict__ ec, int n1c, const T *__restrict__ rhs,
                                                 T *__restrict__ e_dst, const int *__restrict__ skip) {
    const int stop = skip ? *skip : 0;  // tested before the first store (hides the load latency)
    constexpr int TX = VT<D>::TX, TY = VT<D>::TY, TZ = VT<D>::TZ;
    constexpr int HX = TX + 4, HY = TY + 4, HZ = (D == 3) ? TZ + 4 : 1;
    constexpr int NH = HX * HY * HZ;
    __shared__ T e0[NH];
    __shared__ T e1[NH];
    __shared__ T rs[NH];
    const int n1 = L.n1;
    int bx = blockIdx.x, by = blockIdx.y;
    if (D == 2) xcd_tile_2d(bx, by);
    const int gx0 = bx * TX, gy0 = by * TY, gz0 = (D == 3) ? blockIdx.z * TZ : 0;
    const int zoff = (D == 3) ? 2 : 0;
    auto inside = [n1](int x, int y, int z) {
        return x >= 0 && x < n1 && y >= 0 && y < n1 && (D == 2 || (z >= 0 && z < n1));
    };
    // load the step-start iterate over the tile plus a halo of 2, and the
    // right-hand side over the same window; every load of a thread is issued
    // before its first LDS store (one memory round trip)
    constexpr int U = (NH + 255) / 256;
    auto halo_index = [&](int h, int64_t &gi) {
        const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
        const int gx = gx0 + hx - 2, gy = gy0 + hy - 2, gz = gz0 + hz - zoff;
        gi = (int64_t(gz) * n1 + gy) * n1 + gx;
        return inside(gx, gy, gz);
    };
    if (!ec) {
        T v[U], rv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int h = int(threadIdx.x) + u * int(blockDim.x);
            int64_t gi = 0;
            const bool in = h < NH && halo_index(h, gi);
            v[u] = (in && !zero_src) ? e_src[gi] : T(0);
            rv[u] = in ? rhs[gi] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int h = int(threadIdx.x) + u * int(blockDim.x);
            if (h < NH) {
                e0[h] = v[u];
                e1[h] = v[u];
                rs[h] = rv[u];
            }
        }
    } else {
        for (int h = threadIdx.x; h < NH; h += blockDim.x) {
            int64_t gi = 0;
            T v = T(0), rv = T(0);
            if (halo_index(h, gi)) {
                const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
                if (!zero_src) v = e_src[gi];
                v += interp_value<D, T>(ec, n1c, gx0 + hx - 2, gy0 + hy - 2, gz0 + hz - zoff);
                rv = rhs[gi];
            }
            e0[h] = v;
            e1[h] = v;
            rs[h] = rv;
        }
    }
    __syncthreads();
    // red half step on the tile and its halo ring of width 1
    for (int h = threadIdx.x; h < NH; h += blockDim.x) {
        const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
        if (hx < 1 || hx > HX - 2 || hy < 1 || hy > HY - 2) continue;
        if (D == 3 && (hz < 1 || hz > HZ - 2)) continue;
        const int gx = gx0 + hx - 2, gy = gy0 + hy - 2, gz = gz0 + hz - zoff;
        if (!inside(gx, gy, gz) || ((gx + gy + gz) & 1) != 0) continue;
        const int64_t gi = (int64_t(gz) * n1 + gy) * n1 + gx;
        T acc = T(0);
        for (int oz = ((D == 3) ? -1 : 0); oz <= ((D == 3) ? 1 : 0); ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox)
                    acc += coef<D, T>(L, gi, w_of<D>(ox, oy, oz)) * e0[h + (oz * HY + oy) * HX + ox];
        e1[h] = e0[h] + (rs[h] - acc) * inv_diag<D, T>(L, gi);
    }
    __syncthreads();
    if (stop) return;
    // black half step on the tile; write the result
    const int ntile = TX * TY * ((D == 3) ? TZ : 1);
    for (int t = threadIdx.x; t < ntile; t += blockDim.x) {
        const int tx = t % TX, ty = (t / TX) % TY, tz = (D == 3) ? t / (TX * TY) : 0;
        const int gx = gx0 + tx, gy = gy0 + ty, gz = gz0 + tz;
        if (!inside(gx, gy, gz)) continue;
        const int h = ((tz + zoff) * HY + (ty + 2)) * HX + (tx + 2);
        const int64_t gi = (int64_t(gz) * n1 + gy) * n1 + gx;
        T v = e1[h];
        if ((gx + gy + gz) & 1) {
            T acc = T(0);
            for (int oz = ((D == 3) ? -1 : 0); oz <= ((D == 3) ? 1 : 0); ++oz)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int ox = -1; ox <= 1; ++ox)
                        acc += coef<D, T>(L, gi, w_of<D>(ox, oy, oz)) * e1[h + (oz * HY + oy) * HX + ox];
            v = e1[h] + (rs[h] - acc) * inv_diag<D, T>(L, gi);
        }
        e_dst[gi] = v;
    }
}

// --------------------------------------------------------------------------
// NU full red-black steps on a 2-D level in one launch.  The tile of TX x TY
// points is loaded with a halo of H = 2 NU (+2 when RESTRICT); half step j
// updates the points of colour (j & 1) within halo H-1-j from the iterate at
// the start of the half step (two LDS buffers, one barrier per half step), so
// after 2 NU half steps the tile (and, with RESTRICT, a ring of 2 around it)
// holds the smoothed iterate.  The input is (zero_src ? 0 : e_src) + P ec.
// RESTRICT: additionally rc[I] = (P^T (rhs - A e))[I] for the coarse points I
// whose centre child 2I+1 lies in the tile.
// threads of a fused red-black workgroup (tile 32 x 8 plus halo): launches
// with few tiles are latency-bound and take 1024 threads per tile (the halo
// ring's half steps then need one pass), launches with many tiles take 256
// (two instantiations, each compiled for its own register budget)
inline bool rb_wide(int64_t tiles) { return tiles < 1024; }
// levels with at least this many points per direction take 64 x 16 tiles
// (512 threads): the halo ring of a fused step costs about half as much per
// point, and such levels still give thousands of workgroups.  The result of
// every point is the same bits for any tile shape.
constexpr int kRbBigN1 = 1024;
// IGA2L_RB_BIG_N1 in the environment sets another threshold (read at every
// launch: tests send small levels through the large tiles)
inline int rb_big_n1() {
    const char *v = std::getenv("IGA2L_RB_BIG_N1");
    return v ? std::max(1, std::atoi(v)) : kRbBigN1;
}

// The body serves the single-problem kernel and the batched one (tile bx, by).
template <class T, int NU, bool RESTRICT, int TX = 32, int TY = 8>
__device__ __forceinline__ void rb_multi2_body(const LevelDev<T> &L, const T *__restrict__ e_src, int zero_src,
                                               const T *__restrict__ ec, int n1c_interp, const T *__restrict__ rhs,
                                               T *__restrict__ e_dst, T *__restrict__ rc, int n1c,
                                               const int *__restrict__ skip, int bx, int by) {
    static_assert(TX % 2 == 0 && TY % 2 == 0, "whole coarse cells per tile");
    constexpr int H = 2 * NU + (RESTRICT ? 2 : 0);
    constexpr int HX = TX + 2 * H, HY = TY + 2 * H, NH = HX * HY;
    __shared__ T buf[2][NH];
    __shared__ T rs[NH];
    const int stop = skip ? *skip : 0;  // tested before the first store (hides the load latency)
    const int n1 = L.n1;
    const int gx0 = bx * TX, gy0 = by * TY;
    for (int h = threadIdx.x; h < NH; h += blockDim.x) {
        const int hx = h % HX, hy = h / HX;
        const int gx = gx0 + hx - H, gy = gy0 + hy - H;
        T v = T(0), f = T(0);
        if (gx >= 0 && gx < n1 && gy >= 0 && gy < n1) {
            const int64_t gi = int64_t(gy) * n1 + gx;
            if (!zero_src) v = e_src[gi];
            if (ec) v += interp_value<2, T>(ec, n1c_interp, gx, gy, 0);
            f = rhs[gi];
        }
        buf[0][h] = v;
        rs[h] = f;
    }
    __syncthreads();
    int cur = 0;
#pragma unroll
    for (int j = 0; j < 2 * NU; ++j) {
        const int colour = j & 1, halo = H - 1 - j;
        const T *X = buf[cur];
        T *Y = buf[1 - cur];
        for (int h = threadIdx.x; h < NH; h += blockDim.x) {
            const int hx = h % HX, hy = h / HX;
            if (hx < H - halo || hx >= HX - (H - halo) || hy < H - halo || hy >= HY - (H - halo)) continue;
            const int gx = gx0 + hx - H, gy = gy0 + hy - H;
            T v = X[h];
            if (gx >= 0 && gx < n1 && gy >= 0 && gy < n1 && ((gx + gy) & 1) == colour) {
                const int64_t gi = int64_t(gy) * n1 + gx;
                T acc = T(0);
#pragma unroll
                for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                    for (int ox = -1; ox <= 1; ++ox)
                        acc += coef<2, T>(L, gi, w_of<2>(ox, oy, 0)) * X[h + oy * HX + ox];
                v = X[h] + (rs[h] - acc) * inv_diag<2, T>(L, gi);
            }
            Y[h] = v;
        }
        cur = 1 - cur;
        __syncthreads();
    }
    if (stop) return;
    const T *E = buf[cur];
    if constexpr (RESTRICT) {
        // residual on the fine points gx0..gx0+TX, gy0..gy0+TY, kept in the free buffer
        T *R = buf[1 - cur];
        for (int f = threadIdx.x; f < (TX + 1) * (TY + 1); f += blockDim.x) {
            const int fx = f % (TX + 1), fy = f / (TX + 1);
            const int gx = gx0 + fx, gy = gy0 + fy;
            const int h = (fy + H) * HX + (fx + H);
            T r = T(0);
            if (gx < n1 && gy < n1) {
                const int64_t gi = int64_t(gy) * n1 + gx;
                T acc = T(0);
#pragma unroll
                for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                    for (int ox = -1; ox <= 1; ++ox) acc += coef<2, T>(L, gi, w_of<2>(ox, oy, 0)) * E[h + oy * HX + ox];
                r = rs[h] - acc;
            }
            R[f] = r;
        }
        __syncthreads();
        for (int c = threadIdx.x; c < (TX / 2) * (TY / 2); c += blockDim.x) {
            const int cx = c % (TX / 2), cy = c / (TX / 2);
            const int I = gx0 / 2 + cx, J = gy0 / 2 + cy;
            if (I >= n1c || J >= n1c) continue;
            T acc = T(0);
#pragma unroll
            for (int ay = -1; ay <= 1; ++ay)
#pragma unroll
                for (int ax = -1; ax <= 1; ++ax) {
                    const T w = (ax == 0 ? T(1) : T(0.5)) * (ay == 0 ? T(1) : T(0.5));
                    acc += w * R[(2 * cy + 1 + ay) * (TX + 1) + (2 * cx + 1 + ax)];
                }
            rc[int64_t(J) * n1c + I] = acc;
        }
    }
    for (int t = threadIdx.x; t < TX * TY; t += blockDim.x) {
        const int tx = t % TX, ty = t / TX;
        const int gx = gx0 + tx, gy = gy0 + ty;
        if (gx < n1 && gy < n1) e_dst[int64_t(gy) * n1 + gx] = E[(ty + H) * HX + (tx + H)];
    }
}

template <class T, int NU, bool RESTRICT, int NT, int TX = 32, int TY = 8>
__global__ void __launch_bounds__(NT) k_rb_multi2(LevelDev<T> L, const T *__restrict__ e_src, int zero_src,
                                                   const T *__restrict__ ec, int n1c_interp,
                                                   const T *__restrict__ rhs, T *__restrict__ e_dst,
                                                   T *__restrict__ rc, int n1c, const int *__restrict__ skip) {
    int bx, by;
    xcd_tile_2d(bx, by);
    rb_multi2_body<T, NU, RESTRICT, TX, TY>(L, e_src, zero_src, ec, n1c_interp, rhs, e_dst, rc, n1c, skip, bx, by);
}

// batched: pre-smoothing + residual restriction (RESTRICT) or prolongation +
// post-smoothing of level l of every problem of the table
template <class T, int NU, bool RESTRICT, int NT>
__global__ void __launch_bounds__(NT) kb_rb_multi2(const BatchLevel<T> *__restrict__ bl,
                                                    const int2 *__restrict__ map, int zero_src) {
    const int2 m = map[blockIdx.x];
    const BatchLevel<T> &q = bl[m.x];
    int bx, by;
    xcd_relabel(m.y, q.ntx, q.ntx * q.nty, bx, by);
    if constexpr (RESTRICT)
        rb_multi2_body<T, NU, true>(q.L, static_cast<const T *>(nullptr), 1, static_cast<const T *>(nullptr), 0, q.rhs,
                                    q.e_pre, q.rc, q.n1c, q.skip, bx, by);
    else
        rb_multi2_body<T, NU, false>(q.L, q.e_pre, zero_src, q.ecl, q.n1c, q.rhs, q.e_out, static_cast<T *>(nullptr),
                                     0, q.skip, bx, by);
}

// e_dst = e_src + P ec (used only when no post-smoothing step follows)
template <int D, class T>
__global__ void k_interp_add2(const T *__restrict__ e_src, int zero_src, const T *__restrict__ ec, int n1c, int n1,
                              T *__restrict__ e_dst, const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int64_t n = (D == 3) ? int64_t(n1) * n1 * n1 : int64_t(n1) * n1;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ix = int(i % n1), iy = int((i / n1) % n1), iz = (D == 3) ? int(i / (int64_t(n1) * n1)) : 0;
    e_dst[i] = (zero_src ? T(0) : e_src[i]) + interp_value<D, T>(ec, n1c, ix, iy, iz);
}

// rc = P^T (rhs - A e) over tiles of coarse points; the fine residuals of the
// tile's fine region are computed once into LDS.  zero_e: e = 0 (rc = P^T rhs).
template <int D, class T>
__global__ void __launch_bounds__(256) k_res_restrict_tiled(LevelDev<T> L, const T *__restrict__ e, int zero_e,
                                                            const T *__restrict__ rhs, int n1c,
                                                            T *__restrict__ rc, const int *__restrict__ skip) {
    const int stop = skip ? *skip : 0;  // tested before the first store (hides the load latency)
    constexpr int CX = VT<D>::CX, CY = VT<D>::CY, CZ = VT<D>::CZ;
    constexpr int FX = 2 * CX + 1, FY = 2 * CY + 1, FZ = (D == 3) ? 2 * CZ + 1 : 1;  // fine region
    constexpr int EX = FX + 2, EY = FY + 2, EZ = (D == 3) ? FZ + 2 : 1;              // + halo 1
    __shared__ T es[EX * EY * EZ];
    __shared__ T rs[FX * FY * FZ];
    const int n1 = L.n1;
    int bx = blockIdx.x, by = blockIdx.y;
    if (D == 2) xcd_tile_2d(bx, by);
    const int I0 = bx * CX, J0 = by * CY, K0 = (D == 3) ? blockIdx.z * CZ : 0;
    const int fx0 = 2 * I0, fy0 = 2 * J0, fz0 = 2 * K0;  // fine region origin (fine index of child 2I)
    const int ez = (D == 3) ? 1 : 0;
    auto inside = [n1](int x, int y, int z) {
        return x >= 0 && x < n1 && y >= 0 && y < n1 && (D == 2 || (z >= 0 && z < n1));
    };
    // the right-hand side of this thread's fine points and the iterate halo:
    // every load issued before the first LDS store
    constexpr int NF = FX * FY * FZ, UF = (NF + 255) / 256;
    T rv[UF];
#pragma unroll
    for (int u = 0; u < UF; ++u) {
        const int f = int(threadIdx.x) + u * int(blockDim.x);
        const int fx = f % FX, fy = (f / FX) % FY, fz = f / (FX * FY);
        const int gx = fx0 + fx, gy = fy0 + fy, gz = fz0 + fz;
        rv[u] = (f < NF && inside(gx, gy, gz)) ? rhs[(int64_t(gz) * n1 + gy) * n1 + gx] : T(0);
    }
    if (!zero_e) {
        stage_lds<(EX * EY * EZ + 255) / 256, T>(es, EX * EY * EZ, [&](int h) -> T {
            const int hx = h % EX, hy = (h / EX) % EY, hz = h / (EX * EY);
            const int gx = fx0 + hx - 1, gy = fy0 + hy - 1, gz = fz0 + hz - ez;
            return inside(gx, gy, gz) ? e[(int64_t(gz) * n1 + gy) * n1 + gx] : T(0);
        });
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < UF; ++u) {
        const int f = int(threadIdx.x) + u * int(blockDim.x);
        if (f >= NF) continue;
        const int fx = f % FX, fy = (f / FX) % FY, fz = f / (FX * FY);
        const int gx = fx0 + fx, gy = fy0 + fy, gz = fz0 + fz;
        T r = T(0);
        if (inside(gx, gy, gz)) {
            const int64_t gi = (int64_t(gz) * n1 + gy) * n1 + gx;
            r = rv[u];
            if (!zero_e) {
                const int h = ((fz + ez) * EY + (fy + 1)) * EX + (fx + 1);
                T acc = T(0);
                for (int oz = ((D == 3) ? -1 : 0); oz <= ((D == 3) ? 1 : 0); ++oz)
                    for (int oy = -1; oy <= 1; ++oy)
                        for (int ox = -1; ox <= 1; ++ox)
                            acc += coef<D, T>(L, gi, w_of<D>(ox, oy, oz)) * es[h + (oz * EY + oy) * EX + ox];
                r -= acc;
            }
        }
        rs[f] = r;
    }
    __syncthreads();
    if (stop) return;
    const int nct = CX * CY * ((D == 3) ? CZ : 1);
    for (int c = threadIdx.x; c < nct; c += blockDim.x) {
        const int cx = c % CX, cy = (c / CX) % CY, cz = (D == 3) ? c / (CX * CY) : 0;
        const int I = I0 + cx, J = J0 + cy, K = K0 + cz;
        if (I >= n1c || J >= n1c || (D == 3 && K >= n1c)) continue;
        T acc = T(0);
        for (int az = ((D == 3) ? -1 : 0); az <= ((D == 3) ? 1 : 0); ++az)
            for (int ay = -1; ay <= 1; ++ay)
                for (int ax = -1; ax <= 1; ++ax) {
                    const T w = (ax == 0 ? T(1) : T(0.5)) * (ay == 0 ? T(1) : T(0.5)) *
                                ((D == 3 && az != 0) ? T(0.5) : T(1));
                    const int fx = 2 * cx + 1 + ax, fy = 2 * cy + 1 + ay, fz = (D == 3) ? 2 * cz + 1 + az : 0;
                    acc += w * rs[(fz * FY + fy) * FX + fx];
                }
        rc[(int64_t(K) * n1c + J) * n1c + I] = acc;
    }
}

// --------------------------------------------------------------------------
// The tail of the V-cycle (levels lb .. coarsest) in one workgroup.  Every
// level's correction and right-hand side live in LDS on a zero-padded grid
// ((n1+2)^D); the coarsest level is solved with its dense inverse.
constexpr int kBottomThreads = 1024;

template <int D, class T>
struct BottomArgs {
    int nlev;                        // levels handled, lb .. coarsest
    const LevelDev<T> *levels;       // device array, first entry = level lb
};

template <int D>
__device__ __forceinline__ int64_t padded_size(int n1) {
    return (D == 3) ? int64_t(n1 + 2) * (n1 + 2) * (n1 + 2) : int64_t(n1 + 2) * (n1 + 2);
}

// thread layout of the one-workgroup kernel: 32 x 32 (2-D) or 16 x 8 x 8 (3-D)
template <int D>
struct BT;
// one point per thread in 2-D: levels up to 32 x 32 (larger levels run faster
// on the multi-workgroup kernels than as several points per thread here)
template <>
struct BT<2> {
    static constexpr int X = 32, Y = 32, Z = 1;
    static constexpr int KX = 1, KY = 1, KZ = 1;
};
template <>
struct BT<3> {
    static constexpr int X = 16, Y = 8, Z = 8;
    static constexpr int KX = 1, KY = 2, KZ = 2;   // levels up to 16 x 16 x 16
};

// coarsest-level product: Z^{-1} entries each thread loads before the descent
// (registers; the rest of a longer segment is read when it is needed)
template <int D, class T>
struct ZPre {
    // 64 FP32 / 32 FP64 values in 2-D; the 3-D tail owns four points per thread
    static constexpr int K = (D == 2) ? 256 / int(sizeof(T)) : 32 / int(sizeof(T));
};

template <int D, class T>
__device__ __forceinline__ void vcycle_bottom_body(const BottomArgs<D, T> &A, const T *__restrict__ rhs_top,
                                                   T *__restrict__ e_top, int nu1, int nu2,
                                                   const int *__restrict__ skip, unsigned char *smem_raw,
                                                   int nu1_top, int nu2_top) {
    // nu1_top / nu2_top: smoothing steps on the first level handled here
    // (0 for the 2h-coarse correction of aggressive coarsening), nu1 / nu2 below
    if (skip && *skip) return;
    T *sm = reinterpret_cast<T *>(smem_raw);
    // LDS: for each level two correction buffers (a half step reads one and
    // writes the other) and the right-hand side, all padded; then one scratch
    // (level lb's residual, later the coarsest level's flat right-hand side
    // and segment sums).  A padded level of n1 points per direction has pitch
    // n1+2 and the point (x,y,z) at ((z+1)(n1+2) + y+1)(n1+2) + x+1.
    __shared__ int off_e[16][2], off_r[16], s_n1[16], s_cst[16], off_end;
    constexpr int W3 = (D == 3) ? 27 : 9;
    __shared__ T s_c[16][W3];          // constant stencils
    __shared__ T s_cinv[16];
    __shared__ const T *s_S[16];       // per-point stencils / reciprocal diagonals otherwise
    __shared__ const T *s_invd[16];
    __shared__ const T *s_Zinv;
    __shared__ int64_t s_n[16];
    const int tid = threadIdx.x;
    const int tx = tid % BT<D>::X, ty = (tid / BT<D>::X) % BT<D>::Y, tz = (D == 3) ? tid / (BT<D>::X * BT<D>::Y) : 0;
    // level descriptors: one thread per level (independent loads), then the
    // LDS offsets from the staged sizes
    if (tid < A.nlev) {
        const LevelDev<T> &L = A.levels[tid];
        for (int w = 0; w < W3; ++w) s_c[tid][w] = L.c[w];
        s_cinv[tid] = L.cinv;
        s_S[tid] = L.S;
        s_invd[tid] = L.invd;
        s_n[tid] = L.n;
        s_n1[tid] = L.n1;
        s_cst[tid] = L.cst;
        if (tid == A.nlev - 1) s_Zinv = L.Zinv;
    }
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int l = 0; l < A.nlev; ++l) {
            const int n1 = s_n1[l];
            const int ps = (D == 3) ? (n1 + 2) * (n1 + 2) * (n1 + 2) : (n1 + 2) * (n1 + 2);
            off_e[l][0] = acc;
            off_e[l][1] = acc + ps;
            off_r[l] = acc + 2 * ps;
            acc += 3 * ps;
        }
        off_end = acc;
    }
    __syncthreads();
    const int last = A.nlev - 1;
    // the coarsest level's product: thread tid < n nseg takes row i of segment sg
    const int nl1 = s_n1[last];
    const int nz = (D == 3) ? nl1 * nl1 * nl1 : nl1 * nl1;
    const int nseg = max(1, kBottomThreads / nz);
    const int seg_len = (nz + nseg - 1) / nseg;
    const int zi = tid % nz, zsg = tid / nz;
    const int zj0 = zsg * seg_len, zj1 = min(nz, zj0 + seg_len);
    const bool zrow = tid < nz * nseg;
    const T *Zi = s_Zinv;
    constexpr int KZ = ZPre<D, T>::K;
    T zpre[KZ];
#pragma unroll
    for (int k = 0; k < KZ; ++k) zpre[k] = (zrow && zj0 + k < zj1) ? Zi[int64_t(zj0 + k) * nz + zi] : T(0);
    T *scr = sm + off_end;
    {
        const int n1 = s_n1[0];
        const int ps0 = (D == 3) ? (n1 + 2) * (n1 + 2) * (n1 + 2) : (n1 + 2) * (n1 + 2);
        const int total = off_end + max(ps0, nz + kBottomThreads);
        for (int i = tid; i < total; i += kBottomThreads) sm[i] = T(0);
    }
    __syncthreads();
    // loops over the points of a level owned by this thread
#define IGA2L_FOR_POINTS(n1)                                              \
    for (int z = tz; z < ((D == 3) ? (n1) : 1); z += BT<D>::Z)            \
        for (int y = ty; y < (n1); y += BT<D>::Y)                         \
            for (int x = tx; x < (n1); x += BT<D>::X)
    {
        const int n1 = s_n1[0];
        T *r0 = sm + off_r[0];
        IGA2L_FOR_POINTS(n1) {
            const int i = (z * n1 + y) * n1 + x;
            r0[((D == 3) ? ((z + 1) * (n1 + 2) + y + 1) : (y + 1)) * (n1 + 2) + x + 1] = rhs_top[i];
        }
    }
    __syncthreads();
    unsigned cur = 0;   // bit l: buffer of level l holding its current correction
    auto E = [&](int l) { return sm + off_e[l][(cur >> l) & 1]; };
    auto Eo = [&](int l) { return sm + off_e[l][((cur >> l) & 1) ^ 1]; };

    // operator application at padded position c (unpadded index i) of level l
    auto apply = [&](int l, int cst, const T *e, int n1, int c, int i) -> T {
        const int sy = n1 + 2, sz = (n1 + 2) * (n1 + 2);
        T acc = T(0);
        if (cst) {
#pragma unroll
            for (int oz = ((D == 3) ? -1 : 0); oz <= ((D == 3) ? 1 : 0); ++oz)
#pragma unroll
                for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                    for (int ox = -1; ox <= 1; ++ox)
                        acc += s_c[l][w_of<D>(ox, oy, oz)] * e[c + oz * sz + oy * sy + ox];
        } else {
            const T *S = s_S[l];
            const int64_t n = s_n[l];
#pragma unroll
            for (int oz = ((D == 3) ? -1 : 0); oz <= ((D == 3) ? 1 : 0); ++oz)
#pragma unroll
                for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                    for (int ox = -1; ox <= 1; ++ox)
                        acc += S[int64_t(w_of<D>(ox, oy, oz)) * n + i] * e[c + oz * sz + oy * sy + ox];
        }
        return acc;
    };
    // one half step of the given colour on level l: every point of the colour
    // is updated from the iterate at the start of the half step, read from one
    // buffer; the result (updated or copied) goes to the other buffer.  A
    // thread owns the points (tx + X kx, ty + Y ky, tz + Z kz).
    auto half = [&](int l, int colour) {
        const int n1 = s_n1[l], cst = s_cst[l];
        const T cinv = s_cinv[l];
        const T *invd = s_invd[l];
        const T *e = E(l);
        T *eo = Eo(l);
        const T *r = sm + off_r[l];
        constexpr int KX = BT<D>::KX, KY = BT<D>::KY, KZ = BT<D>::KZ;
#pragma unroll
        for (int k = 0; k < KX * KY * KZ; ++k) {
            const int x = tx + BT<D>::X * (k % KX), y = ty + BT<D>::Y * ((k / KX) % KY),
                      z = (D == 3) ? tz + BT<D>::Z * (k / (KX * KY)) : 0;
            if (x < n1 && y < n1 && (D == 2 || z < n1)) {
                const int c = ((D == 3) ? ((z + 1) * (n1 + 2) + y + 1) : (y + 1)) * (n1 + 2) + x + 1;
                T v = e[c];
                if (((x + y + z) & 1) == colour) {
                    const int i = (z * n1 + y) * n1 + x;
                    const T id = cst ? cinv : invd[i];
                    v = e[c] + (r[c] - apply(l, cst, e, n1, c, i)) * id;
                }
                eo[c] = v;
            }
        }
        __syncthreads();
        cur ^= 1u << l;
    };

    for (int l = 0; l < last; ++l) {
        for (int k = 0; k < (l == 0 ? nu1_top : nu1); ++k) {
            half(l, 0);
            half(l, 1);
        }
        const int n1 = s_n1[l], cst = s_cst[l];
        const T *e = E(l);
        const T *r = sm + off_r[l];
        IGA2L_FOR_POINTS(n1) {
            const int i = (z * n1 + y) * n1 + x;
            const int c = ((D == 3) ? ((z + 1) * (n1 + 2) + y + 1) : (y + 1)) * (n1 + 2) + x + 1;
            scr[c] = r[c] - apply(l, cst, e, n1, c, i);
        }
        __syncthreads();
        const int n1c = s_n1[l + 1];
        T *rc = sm + off_r[l + 1];
        T *ecl = E(l + 1);
        IGA2L_FOR_POINTS(n1c) {
            T acc = T(0);
            for (int az = ((D == 3) ? -1 : 0); az <= ((D == 3) ? 1 : 0); ++az)
                for (int ay = -1; ay <= 1; ++ay)
                    for (int ax = -1; ax <= 1; ++ax) {
                        const int fx = 2 * x + 1 + ax, fy = 2 * y + 1 + ay, fz = (D == 3) ? 2 * z + 1 + az : 0;
                        // the scratch is shared by all levels: never read outside level l's points
                        if (fx >= n1 || fy >= n1 || (D == 3 && fz >= n1)) continue;
                        const T w = (ax == 0 ? T(1) : T(0.5)) * (ay == 0 ? T(1) : T(0.5)) *
                                    ((D == 3 && az != 0) ? T(0.5) : T(1));
                        acc += w * scr[((D == 3) ? ((fz + 1) * (n1 + 2) + fy + 1) : (fy + 1)) * (n1 + 2) + fx + 1];
                    }
            const int cc = ((D == 3) ? ((z + 1) * (n1c + 2) + y + 1) : (y + 1)) * (n1c + 2) + x + 1;
            rc[cc] = acc;
            ecl[cc] = T(0);
        }
        __syncthreads();
    }
    {
        // coarsest level: e = Z^{-1} r.  The right-hand side is copied to a flat
        // array; each row's dot product is split into nseg segments handled by
        // different threads (Z^{-1} is symmetric: row i is read as column i, so
        // consecutive threads read consecutive words), then summed in LDS.
        const int n1 = nl1;
        const T *r = sm + off_r[last];
        T *e = E(last);
        T *rflat = scr;
        T *part = scr + nz;
        for (int i = tid; i < nz; i += kBottomThreads) {
            const int x = i % n1, y = (i / n1) % n1, z = (D == 3) ? i / (n1 * n1) : 0;
            rflat[i] = r[((D == 3) ? ((z + 1) * (n1 + 2) + y + 1) : (y + 1)) * (n1 + 2) + x + 1];
        }
        __syncthreads();
        if (zrow) {
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < KZ; ++k)
                if (zj0 + k < zj1) acc += zpre[k] * rflat[zj0 + k];
#pragma unroll 16
            for (int j = zj0 + KZ; j < zj1; ++j) acc += Zi[int64_t(j) * nz + zi] * rflat[j];
            if (nseg == 1) {
                const int x = zi % n1, y = (zi / n1) % n1, z = (D == 3) ? zi / (n1 * n1) : 0;
                e[((D == 3) ? ((z + 1) * (n1 + 2) + y + 1) : (y + 1)) * (n1 + 2) + x + 1] = acc;
            } else {
                part[zsg * nz + zi] = acc;
            }
        }
        __syncthreads();
        if (nseg > 1) {
            for (int i = tid; i < nz; i += kBottomThreads) {
                T acc = T(0);
                for (int sg = 0; sg < nseg; ++sg) acc += part[sg * nz + i];
                const int x = i % n1, y = (i / n1) % n1, z = (D == 3) ? i / (n1 * n1) : 0;
                e[((D == 3) ? ((z + 1) * (n1 + 2) + y + 1) : (y + 1)) * (n1 + 2) + x + 1] = acc;
            }
        }
        __syncthreads();
    }
    for (int l = last - 1; l >= 0; --l) {
        const int n1 = s_n1[l], n1c = s_n1[l + 1];
        T *e = E(l);
        const T *ecl = E(l + 1);
        IGA2L_FOR_POINTS(n1) {
            int Ix[2], Iy[2], Iz[2];
            T wx[2], wy[2], wz[2];
            const int nx = parents<T>(x, n1c, Ix, wx), ny = parents<T>(y, n1c, Iy, wy);
            int nzp = 1;
            Iz[0] = 0;
            wz[0] = T(1);
            if (D == 3) nzp = parents<T>(z, n1c, Iz, wz);
            T acc = T(0);
            for (int cc = 0; cc < nzp; ++cc)
                for (int bb = 0; bb < ny; ++bb)
                    for (int aa = 0; aa < nx; ++aa) {
                        const int q = ((D == 3) ? ((Iz[cc] + 1) * (n1c + 2) + Iy[bb] + 1) : (Iy[bb] + 1)) * (n1c + 2) +
                                      Ix[aa] + 1;
                        acc += wz[cc] * wy[bb] * wx[aa] * ecl[q];
                    }
            e[((D == 3) ? ((z + 1) * (n1 + 2) + y + 1) : (y + 1)) * (n1 + 2) + x + 1] += acc;
        }
        __syncthreads();
        for (int k = 0; k < (l == 0 ? nu2_top : nu2); ++k) {
            half(l, 0);
            half(l, 1);
        }
    }
    {
        const int n1 = s_n1[0];
        const T *e0 = E(0);
        IGA2L_FOR_POINTS(n1) {
            e_top[(z * n1 + y) * n1 + x] = e0[((D == 3) ? ((z + 1) * (n1 + 2) + y + 1) : (y + 1)) * (n1 + 2) + x + 1];
        }
    }
#undef IGA2L_FOR_POINTS
}

template <int D, class T>
__global__ void __launch_bounds__(kBottomThreads) k_vcycle_bottom(BottomArgs<D, T> A, const T *__restrict__ rhs_top,
                                                                  T *__restrict__ e_top, int nu1, int nu2,
                                                                  const int *__restrict__ skip, int nu1_top,
                                                                  int nu2_top) {
    extern __shared__ unsigned char smem_raw[];
    vcycle_bottom_body<D, T>(A, rhs_top, e_top, nu1, nu2, skip, smem_raw, nu1_top, nu2_top);
}

// batched: one workgroup per problem of the table
template <class T>
__global__ void __launch_bounds__(kBottomThreads) kb_vcycle_bottom(const BatchBottom<T> *__restrict__ bb, int nu1,
                                                                   int nu2) {
    extern __shared__ unsigned char smem_raw[];
    const BatchBottom<T> &q = bb[blockIdx.x];
    const BottomArgs<2, T> a{q.nlev, q.levels};
    vcycle_bottom_body<2, T>(a, q.rhs, q.e, nu1, nu2, q.skip, smem_raw, nu1, nu2);
}

template <class T>
size_t bottom_level(const Problem &P) {
    return std::is_same<T, double>::value ? P.vc_bottom64 : P.vc_bottom32;
}

template <class T>
const LevelDev<T> *levdev(const Problem &P) {
    return std::is_same<T, double>::value ? reinterpret_cast<const LevelDev<T> *>(P.levdev64.ptr)
                                          : reinterpret_cast<const LevelDev<T> *>(P.levdev32.ptr);
}

template <class T>
LevelDev<T> levhost(const Problem &P, size_t l) {
    if constexpr (std::is_same<T, double>::value) return P.levhost64[l];
    else return P.levhost32[l];
}

template <int D, class T>
void vcycle_top(Problem &P, size_t l, const T *rhs, T *e_out, int nu1, int nu2, hipStream_t s, int nu1_here = -1,
                int nu2_here = -1);

template <class T, int NU, bool RESTRICT>
void launch_rb_multi2(const Problem &P, const LevelDev<T> &Ld, const T *e_src, bool zero_src, const T *ec,
                      int n1c_interp, const T *rhs, T *e_dst, T *rc, int n1c, hipStream_t s) {
    if constexpr (NU <= 2) if (Ld.n1 >= rb_big_n1()) {
        // large levels: 64 x 16 tiles, about half the halo work per point of 32 x 8
        // (up to two steps: the LDS of the tile and its halo stays under 64 KB)
        const dim3 grid(nblk(Ld.n1, 64), nblk(Ld.n1, 16), 1);
        hipLaunchKernelGGL((k_rb_multi2<T, NU, RESTRICT, 512, 64, 16>), grid, dim3(512), 0, s, Ld, e_src,
                           zero_src ? 1 : 0, ec, n1c_interp, rhs, e_dst, rc, n1c, P.skip);
        return;
    }
    const dim3 grid(nblk(Ld.n1, 32), nblk(Ld.n1, 8), 1);
    if (rb_wide(grid.x * grid.y))
        hipLaunchKernelGGL((k_rb_multi2<T, NU, RESTRICT, 1024>), grid, dim3(1024), 0, s, Ld, e_src, zero_src ? 1 : 0,
                           ec, n1c_interp, rhs, e_dst, rc, n1c, P.skip);
    else
        hipLaunchKernelGGL((k_rb_multi2<T, NU, RESTRICT, 256>), grid, dim3(256), 0, s, Ld, e_src, zero_src ? 1 : 0,
                           ec, n1c_interp, rhs, e_dst, rc, n1c, P.skip);
}

template <class T, bool RESTRICT>
void rb_multi2(const Problem &P, int nu, const LevelDev<T> &Ld, const T *e_src, bool zero_src, const T *ec,
               int n1c_interp, const T *rhs, T *e_dst, T *rc, int n1c, hipStream_t s) {
    switch (nu) {
        case 0: launch_rb_multi2<T, 0, RESTRICT>(P, Ld, e_src, zero_src, ec, n1c_interp, rhs, e_dst, rc, n1c, s); break;
        case 1: launch_rb_multi2<T, 1, RESTRICT>(P, Ld, e_src, zero_src, ec, n1c_interp, rhs, e_dst, rc, n1c, s); break;
        case 2: launch_rb_multi2<T, 2, RESTRICT>(P, Ld, e_src, zero_src, ec, n1c_interp, rhs, e_dst, rc, n1c, s); break;
        case 3: launch_rb_multi2<T, 3, RESTRICT>(P, Ld, e_src, zero_src, ec, n1c_interp, rhs, e_dst, rc, n1c, s); break;
        case 4: launch_rb_multi2<T, 4, RESTRICT>(P, Ld, e_src, zero_src, ec, n1c_interp, rhs, e_dst, rc, n1c, s); break;
        default: throw Error{IGA2L_EUNSUPPORTED, "fused red-black steps support nu <= 4"};
    }
}

// 2-D top level: pre-smoothing + residual + restriction in one launch, the
// coarser levels, then prolongation + post-smoothing in one launch
template <class T>
void vcycle_top_fused2(Problem &P, size_t l, const T *rhs, T *e_out, int nu1, int nu2, hipStream_t s) {
    Level &L = P.levels[l];
    Level &C = P.levels[l + 1];
    const LevelDev<T> Ld = levhost<T>(P, l);
    const int n1c = C.g.n1;
    T *epre = L.e[0].as<T>();
    T *rc = C.rhs.as<T>();
    T *ecl = C.res.as<T>();
    rb_multi2<T, true>(P, nu1, Ld, static_cast<const T *>(nullptr), true, static_cast<const T *>(nullptr), 0, rhs,
                       epre, rc, n1c, s);
    vcycle_top<2, T>(P, l + 1, rc, ecl, nu1, nu2, s);
    rb_multi2<T, false>(P, nu2, Ld, epre, nu1 == 0, ecl, n1c, rhs, e_out, static_cast<T *>(nullptr), 0, s);
}

// V-cycle from zero on level l of the multi-workgroup part; result in e_out.
// nu1_here / nu2_here (if >= 0): smoothing steps on level l itself, nu1 / nu2
// on the coarser levels
template <int D, class T>
void vcycle_top(Problem &P, size_t l, const T *rhs, T *e_out, int nu1, int nu2, hipStream_t s, int nu1_here,
                int nu2_here) {
    const int n1h = nu1_here >= 0 ? nu1_here : nu1, n2h = nu2_here >= 0 ? nu2_here : nu2;
    const size_t lb = bottom_level<T>(P);
    if (l == lb) {
        const size_t nlev = P.levels.size() - lb;
        BottomArgs<D, T> a{int(nlev), levdev<T>(P) + lb};
        const size_t shm = size_t(vcycle_bottom_lds(P, lb)) * sizeof(T);
        hipLaunchKernelGGL((k_vcycle_bottom<D, T>), dim3(1), dim3(kBottomThreads), shm, s, a, rhs, e_out, nu1, nu2,
                           P.skip, n1h, n2h);
        return;
    }
    Level &L = P.levels[l];
    Level &C = P.levels[l + 1];
    const LevelDev<T> Ld = levhost<T>(P, l);
    const int n1 = L.g.n1, n1c = C.g.n1;
    if constexpr (D == 2) {
        if (n1h == nu1 && n2h == nu2 && nu1 <= 4 && nu2 <= 4 && nu2 >= 1) {
            vcycle_top_fused2<T>(P, l, rhs, e_out, nu1, nu2, s);
            return;
        }
    }
    using TS = VT<D>;
    const dim3 sgrid(nblk(n1, TS::TX), nblk(n1, TS::TY), D == 3 ? nblk(n1, TS::TZ) : 1);
    const dim3 rgrid(nblk(n1c, TS::CX), nblk(n1c, TS::CY), D == 3 ? nblk(n1c, TS::CZ) : 1);
    T *buf[2] = {L.e[0].as<T>(), L.e[1].as<T>()};
    int cur = 0;
    bool zero = true;
    for (int k = 0; k < n1h; ++k) {
        hipLaunchKernelGGL((k_rb_step<D, T>), sgrid, dim3(256), 0, s, Ld, buf[cur], zero ? 1 : 0,
                           static_cast<const T *>(nullptr), 0, rhs, buf[1 - cur], P.skip);
        cur = 1 - cur;
        zero = false;
    }
    T *rc = C.rhs.as<T>();
    T *ecl = C.res.as<T>();
    hipLaunchKernelGGL((k_res_restrict_tiled<D, T>), rgrid, dim3(256), 0, s, Ld, buf[cur], zero ? 1 : 0, rhs, n1c, rc,
                       P.skip);
    vcycle_top<D, T>(P, l + 1, rc, ecl, nu1, nu2, s);
    // post-smoothing; the first step loads e + P ec, the last one writes e_out
    if (n2h == 0) {
        hipLaunchKernelGGL((k_interp_add2<D, T>), dim3(nblk(L.g.n, 256)), dim3(256), 0, s, buf[cur], zero ? 1 : 0,
                           static_cast<const T *>(ecl), n1c, n1, e_out, P.skip);
        return;
    }
    for (int k = 0; k < n2h; ++k) {
        T *dst = (k == n2h - 1) ? e_out : buf[1 - cur];
        hipLaunchKernelGGL((k_rb_step<D, T>), sgrid, dim3(256), 0, s, Ld, buf[cur], zero ? 1 : 0,
                           (k == 0) ? static_cast<const T *>(ecl) : static_cast<const T *>(nullptr), n1c, rhs, dst,
                           P.skip);
        cur = 1 - cur;
        zero = false;
    }
}

}  // namespace

template <class T>
void launch_vcycle(Problem &P, const T *rhs, T *e, int nu1, int nu2, hipStream_t s) {
    IGA2L_REQUIRE(P.vcycle_ready, IGA2L_EINVAL, "V-cycle hierarchy not set up");
    if (P.dim == 2) vcycle_top<2, T>(P, 0, rhs, e, nu1, nu2, s);
    else vcycle_top<3, T>(P, 0, rhs, e, nu1, nu2, s);
}
template void launch_vcycle<double>(Problem &, const double *, double *, int, int, hipStream_t);
template void launch_vcycle<float>(Problem &, const float *, float *, int, int, hipStream_t);

// Aggressive coarsening (the coarse level is degree 1 on 2h): e = P_0 C P_0^T d
// with P_0 the linear interpolation of the hierarchy from level 1 to level 0.
// exact: C = the DST-I solve of level 1 (FP64); otherwise C = one V(nu1,nu2)
// cycle from zero on levels 1, 2, ..., i.e. a V-cycle from level 0 without
// smoothing on level 0.
template <int D, class T>
static void coarse_aggressive_dim(Problem &P, const T *d, T *e, bool exact, int nu1, int nu2, hipStream_t s) {
    if (!exact) {
        vcycle_top<D, T>(P, 0, d, e, nu1, nu2, s, 0, 0);
        return;
    }
    IGA2L_REQUIRE(P.agg_direct_ready, IGA2L_EINVAL, "exact 2h solve not set up (setup_blocks with aggressive)");
    Level &L = P.levels[0];
    Level &C = P.levels[1];
    const LevelDev<T> Ld = levhost<T>(P, 0);
    const int n1 = L.g.n1, n1c = C.g.n1;
    const int64_t n2 = C.g.n;
    using TS = VT<D>;
    const dim3 rgrid(nblk(n1c, TS::CX), nblk(n1c, TS::CY), D == 3 ? nblk(n1c, TS::CZ) : 1);
    double *rc64 = P.agg64.as<double>(), *ec64 = rc64 + n2, *t1 = rc64 + 2 * n2;
    T *rc = C.rhs.as<T>(), *ecl = C.res.as<T>();
    hipLaunchKernelGGL((k_res_restrict_tiled<D, T>), rgrid, dim3(256), 0, s, Ld, static_cast<const T *>(nullptr), 1,
                       d, n1c, rc, P.skip);
    if constexpr (std::is_same<T, double>::value) {
        dst_apply_2h(P, rc, ecl, t1, s);
    } else {
        launch_convert(rc, rc64, n2, false, s, P.skip);
        dst_apply_2h(P, rc64, ec64, t1, s);
        launch_convert(ec64, ecl, n2, true, s, P.skip);
    }
    hipLaunchKernelGGL((k_interp_add2<D, T>), dim3(nblk(L.g.n, 256)), dim3(256), 0, s, static_cast<const T *>(nullptr),
                       1, static_cast<const T *>(ecl), n1c, n1, e, P.skip);
}

template <class T>
void launch_coarse_aggressive(Problem &P, const T *d, T *e, bool exact, int nu1, int nu2, hipStream_t s) {
    IGA2L_REQUIRE(P.vcycle_ready && P.levels.size() >= 2, IGA2L_EUNSUPPORTED,
                  "aggressive coarsening needs a V-cycle hierarchy with a 2h level (more than 512 coarse unknowns)");
    if (P.dim == 2) coarse_aggressive_dim<2, T>(P, d, e, exact, nu1, nu2, s);
    else coarse_aggressive_dim<3, T>(P, d, e, exact, nu1, nu2, s);
}
template void launch_coarse_aggressive<double>(Problem &, const double *, double *, bool, int, int, hipStream_t);
template void launch_coarse_aggressive<float>(Problem &, const float *, float *, bool, int, int, hipStream_t);

// LDS (in elements) the bottom kernel needs for levels lb..coarsest
int64_t vcycle_bottom_lds(const Problem &P, size_t lb) {
    auto ps = [&](int n1) {
        int64_t r = 1;
        for (int k = 0; k < P.dim; ++k) r *= (n1 + 2);
        return r;
    };
    int64_t tot = 0;
    for (size_t l = lb; l < P.levels.size(); ++l) tot += 3 * ps(P.levels[l].g.n1);
    // scratch: level lb's residual, or the coarsest level's flat right-hand side
    // and its segment sums (at most kBottomThreads of them)
    const int n1c = P.levels.back().g.n1;
    int64_t nz = 1;
    for (int k = 0; k < P.dim; ++k) nz *= n1c;
    return tot + std::max<int64_t>(ps(P.levels[lb].g.n1), nz + kBottomThreads);
}

// points one thread owns in the bottom kernel (strided 32x32 or 16x8x8 layout)
bool vcycle_bottom_fits(const Problem &P, size_t lb) {
    const int n1 = P.levels[lb].g.n1;
    bool ok;
    if (P.dim == 2) ok = n1 <= BT<2>::X * BT<2>::KX && n1 <= BT<2>::Y * BT<2>::KY;
    else ok = n1 <= BT<3>::X * BT<3>::KX && n1 <= BT<3>::Y * BT<3>::KY && n1 <= BT<3>::Z * BT<3>::KZ;
    return ok && P.levels.size() - lb <= 16;
}

// ------------------------------------------------------- batched launchers --
template <class T>
void launch_rb_multi2_batch(const BatchLevel<T> *bl, const int2 *map, int nwg, int nu, bool restrict_, bool zero_src,
                            hipStream_t s) {
    auto go = [&](auto kern, unsigned nt) {
        hipLaunchKernelGGL(kern, dim3(nwg), dim3(nt), 0, s, bl, map, zero_src ? 1 : 0);
    };
    const bool wide = rb_wide(nwg);
#define IGA2L_RBB(NU)                                                                        \
    case NU:                                                                                 \
        if (restrict_) {                                                                     \
            if (wide) go(kb_rb_multi2<T, NU, true, 1024>, 1024);                             \
            else go(kb_rb_multi2<T, NU, true, 256>, 256);                                    \
        } else {                                                                             \
            if (wide) go(kb_rb_multi2<T, NU, false, 1024>, 1024);                            \
            else go(kb_rb_multi2<T, NU, false, 256>, 256);                                   \
        }                                                                                    \
        break;
    switch (nu) {
        IGA2L_RBB(0)
        IGA2L_RBB(1)
        IGA2L_RBB(2)
        IGA2L_RBB(3)
        IGA2L_RBB(4)
        default: throw Error{IGA2L_EUNSUPPORTED, "fused red-black steps support nu <= 4"};
    }
#undef IGA2L_RBB
}
template void launch_rb_multi2_batch<double>(const BatchLevel<double> *, const int2 *, int, int, bool, bool,
                                             hipStream_t);
template void launch_rb_multi2_batch<float>(const BatchLevel<float> *, const int2 *, int, int, bool, bool,
                                            hipStream_t);

template <class T>
void launch_vcycle_bottom_batch(const BatchBottom<T> *bb, int nprob, size_t shm, int nu1, int nu2, hipStream_t s) {
    hipLaunchKernelGGL((kb_vcycle_bottom<T>), dim3(nprob), dim3(kBottomThreads), shm, s, bb, nu1, nu2);
}
template void launch_vcycle_bottom_batch<double>(const BatchBottom<double> *, int, size_t, int, int, hipStream_t);
template void launch_vcycle_bottom_batch<float>(const BatchBottom<float> *, int, size_t, int, int, hipStream_t);

}  // namespace iga2l
