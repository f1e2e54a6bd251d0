// kernels_fine.hip -- fine-level kernels of the two-level solver on gfx950:
// the wide-band residual (symmetric padded-diagonal operator, LDS-staged halo
// of width p), the coloured overlapping multiplicative Schwarz step, the
// lexicographic (hyperplane) Schwarz step, the batched inversion of the
// Schwarz block matrices and the deterministic residual norm.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "internal.h"

namespace iga2l {

namespace {

constexpr int kWave = 64;
// at most 512 threads per Schwarz tile: 256 VGPRs per lane, no spills for 7x7 blocks
constexpr int kColourThreads = 512;
// grids below this many unknowns take the register-prefetching Schwarz kernel
constexpr int64_t kColourPreMaxN = int64_t(1) << 19;

__host__ __device__ constexpr int cpow(int b, int e) { return e == 0 ? 1 : b * cpow(b, e - 1); }

// ------------------------------------------------------------------------
// Operator entry A[i][i+o] from the symmetric padded-diagonal form.
// padi = padded position of row i; w = offset index of o (x fastest, each
// component shifted by P); delta = padded shift of o.
template <int D, int P, class T>
__device__ __forceinline__ T dia_entry(const T *__restrict__ val, int64_t npad, int64_t padi, int w, int64_t delta) {
    constexpr int W = cpow(2 * P + 1, D);
    constexpr int c0 = (W - 1) / 2;
    if (w >= c0) return val[int64_t(w - c0) * npad + padi];
    return val[int64_t(c0 - w) * npad + padi + delta];
}

// ------------------------------------------------------------------------
// Interior rows of the kappa = 1 operator are translation invariant: rows whose
// coordinates all lie in [ulo, uhi] carry the (2p+1)^d stencil cs (bit for
// bit: the interior element matrices are one copy).  Such rows read cs
// (uniform addresses) instead of the diagonals.
__device__ __forceinline__ bool point_uniform(int x, int y, int z, int ulo, int uhi, int dim) {
    return x >= ulo && x <= uhi && y >= ulo && y <= uhi && (dim == 2 || (z >= ulo && z <= uhi));
}

// ------------------------------------------------------------------------
// kappa = 1 in 3-D: the operator is K1 (x) M1 (x) M1 + M1 (x) K1 (x) M1 +
// M1 (x) M1 (x) K1.  The entry for offsets (ox, oy, oz) from the 1-D factor
// entries of the point's rows, with the products and sums grouped and
// rounded as in the assembly of the diagonals (contraction off, every
// operation rounded on its own), so it equals the stored diagonal bit for
// bit: kx (my mz) + mx (ky mz) + mx (my kz), the yz products (myz, kymz,
// mykz) formed once per stencil row.  Out-of-grid neighbours give 0.
__device__ __forceinline__ double kron3_entry(double kx, double mx, double myz, double kymz, double mykz) {
#pragma clang fp contract(off)
    const double p0 = kx * myz;
    const double p1 = mx * kymz;
    const double p2 = mx * mykz;
    double t = 0.0;
    t += p0;
    t += p1;
    t += p2;
    return t;
}

// 3-D row of a point next to the boundary from the 1-D factors (K then M,
// [n1][2P+1] each), accumulated against the LDS halo in the diagonal order.
// FP64: the entries equal the stored diagonals bit for bit.  FP32 (the
// correction cycle): FP32 factors, the sum regrouped as

// A row of a 2-D operator that is a tensor sum of direction-dependent 1-D
// factors, A = Kx (x) My + Mx (x) Ky (the quarter annulus: fac holds the rows
// of Kx, Mx, Ky, My, each [n1][2P+1]), applied by sum factorisation: per
// stencil row the x sums of both x factors, then the y weights.  The factor
// rows of a point next to the boundary are zero beyond the grid.
template <int P, class T>
__device__ __forceinline__ T fac2_row_dot(const T *__restrict__ fac, int n1, int gx, int gy, const T *xs, int lc,
                                         int HX) {
    constexpr int W1 = 2 * P + 1;
    const int64_t nw = int64_t(n1) * W1;
    const T *Kx = fac + int64_t(gx) * W1, *Mx = fac + nw + int64_t(gx) * W1;
    const T *Ky = fac + 2 * nw + int64_t(gy) * W1, *My = fac + 3 * nw + int64_t(gy) * W1;
    T acc = T(0);
#pragma unroll
    for (int oy = -P; oy <= P; ++oy) {
        T kx = T(0), mx = T(0);
#pragma unroll
        for (int ox = -P; ox <= P; ++ox) {
            const T v = xs[lc + oy * HX + ox];
            kx += Kx[ox + P] * v;
            mx += Mx[ox + P] * v;
        }
        acc += My[oy + P] * kx + Ky[oy + P] * mx;
    }
    return acc;
}

// kx (my mz) + mx (ky mz + my kz), the yz part formed once per stencil row.
template <int P, class T>
__device__ __forceinline__ T kron3_row_dot(const T *__restrict__ kron, int n1, int gx, int gy, int gz, const T *xs,
                                           int lc, int HX, int HY) {
    constexpr int W1 = 2 * P + 1;
    const T *K = kron, *M = kron + int64_t(n1) * W1;
    // the x rows stay in registers; the y and z loops stay rolled (register budget)
    T kx[W1], mx[W1];
#pragma unroll
    for (int o = 0; o < W1; ++o) {
        kx[o] = K[gx * W1 + o];
        mx[o] = M[gx * W1 + o];
    }
    T acc = T(0);
#pragma unroll 1
    for (int oz = -P; oz <= P; ++oz) {
        const T kz = K[gz * W1 + oz + P], mz = M[gz * W1 + oz + P];
#pragma unroll 1
        for (int oy = -P; oy <= P; ++oy) {
            const T ky = K[gy * W1 + oy + P], my = M[gy * W1 + oy + P];
            const T *xr = xs + lc + (oz * HY + oy) * HX;
            if constexpr (std::is_same<T, double>::value) {
                const double myz = my * mz, kymz = ky * mz, mykz = my * kz;
#pragma unroll
                for (int ox = -P; ox <= P; ++ox)
                    acc += kron3_entry(kx[ox + P], mx[ox + P], myz, kymz, mykz) * xr[ox];
            } else {
                const T a = my * mz, c = ky * mz + my * kz;
#pragma unroll
                for (int ox = -P; ox <= P; ++ox) acc += (kx[ox + P] * a + mx[ox + P] * c) * xr[ox];
            }
        }
    }
    return acc;
}

// Residual r = b - A x over tiles of TX x TY (x TZ) points; x staged in LDS
// with a halo of width P (zeros outside the grid).  NORM: the per-workgroup
// sums of r^2 are combined by the last workgroup to finish, in a fixed
// order, into ||r||_2 and the scaling of the FP32 correction cycle.
// The body serves the single-problem kernel and the batched one: tile
// (bx, by, bz), its partial sum goes to *part, xs = LDS of the halo tile.
template <int D, int P, class T, bool NORM>
__device__ __forceinline__ void residual_body(const T *__restrict__ val, int64_t npad, int pitch1, int pitch2, int n1,
                                              int TX, int TY, int TZ, const T *__restrict__ x,
                                              const T *__restrict__ b, T *__restrict__ r, double *__restrict__ part,
                                              const T *__restrict__ cs, int ulo, int uhi,
                                              const int *__restrict__ skip, int bx, int by, int bz, T *xs,
                                              const T *__restrict__ kron = nullptr) {
    const int stop = skip ? *skip : 0;  // tested before the first store (hides the load latency)
    const int HX = TX + 2 * P, HY = TY + 2 * P, HZ = (D == 3) ? TZ + 2 * P : 1;
    const int gx0 = bx * TX, gy0 = by * TY, gz0 = (D == 3) ? bz * TZ : 0;
    const int nh = HX * HY * HZ;
    const int t = threadIdx.x;
    const int tx = t % TX, ty = (t / TX) % TY, tz = (D == 3) ? t / (TX * TY) : 0;
    const int gx = gx0 + tx, gy = gy0 + ty, gz = gz0 + tz;
    const bool active = t < TX * TY * ((D == 3) ? TZ : 1) && gx < n1 && gy < n1 && (D == 2 || gz < n1);
    const int64_t gi = active ? (int64_t(gz) * n1 + gy) * n1 + gx : 0;
    const T bv = active ? b[gi] : T(0);   // issued with the halo loads
    // the interior stencil (kappa = 1) staged in LDS behind the halo
    constexpr int W = cpow(2 * P + 1, D);
    T *css = xs + nh;
    if (cs)
        for (int w = threadIdx.x; w < W; w += blockDim.x) css[w] = cs[w];
    for (int h = threadIdx.x; h < nh; h += blockDim.x) {
        int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
        int hgx = gx0 + hx - P, hgy = gy0 + hy - P, hgz = (D == 3) ? gz0 + hz - P : 0;
        bool in = hgx >= 0 && hgx < n1 && hgy >= 0 && hgy < n1 && (D == 2 || (hgz >= 0 && hgz < n1));
        xs[h] = in ? x[(int64_t(hgz) * n1 + hgy) * n1 + hgx] : T(0);
    }
    __syncthreads();
    // a wavefront whose rows all carry the interior stencil reads it instead of
    // the diagonals (one path per wavefront; only wavefronts touching the rows
    // next to the grid boundary read the operator)
    const bool uni = cs != nullptr && __all(!active || point_uniform(gx, gy, gz, ulo, uhi, D));
    double rr = 0.0;
    if (active) {
        const int64_t padi = int64_t(gx + P) + int64_t(gy + P) * pitch1 + ((D == 3) ? int64_t(gz + P) * pitch2 : 0);
        const int lc = ((tz + ((D == 3) ? P : 0)) * HY + (ty + P)) * HX + (tx + P);
        T acc = T(0);
        if constexpr (D == 2) {
            if (uni) {
#pragma unroll
                for (int oy = -P; oy <= P; ++oy)
#pragma unroll
                    for (int ox = -P; ox <= P; ++ox)
                        acc += css[(oy + P) * (2 * P + 1) + (ox + P)] * xs[lc + oy * HX + ox];
            } else if (kron) {
                acc = fac2_row_dot<P, T>(kron, n1, gx, gy, xs, lc, HX);
            } else {
#pragma unroll
                for (int oy = -P; oy <= P; ++oy)
#pragma unroll
                    for (int ox = -P; ox <= P; ++ox) {
                        const int w = (oy + P) * (2 * P + 1) + (ox + P);
                        const T a = dia_entry<D, P, T>(val, npad, padi, w, int64_t(ox) + int64_t(oy) * pitch1);
                        acc += a * xs[lc + oy * HX + ox];
                    }
            }
        } else {
            // 3-D: the z loop stays rolled (a fully unrolled (2p+1)^3 body holds too many registers)
            if (uni) {
#pragma unroll 1
                for (int oz = -P; oz <= P; ++oz)
#pragma unroll
                    for (int oy = -P; oy <= P; ++oy)
#pragma unroll
                        for (int ox = -P; ox <= P; ++ox)
                            acc += css[((oz + P) * (2 * P + 1) + (oy + P)) * (2 * P + 1) + (ox + P)] *
                                   xs[lc + (oz * HY + oy) * HX + ox];
            } else if (kron) {
                acc = kron3_row_dot<P, T>(kron, n1, gx, gy, gz, xs, lc, HX, HY);
            } else {
#pragma unroll 1
                for (int oz = -P; oz <= P; ++oz)
#pragma unroll
                    for (int oy = -P; oy <= P; ++oy)
#pragma unroll
                        for (int ox = -P; ox <= P; ++ox) {
                            const int w = ((oz + P) * (2 * P + 1) + (oy + P)) * (2 * P + 1) + (ox + P);
                            const T a = dia_entry<D, P, T>(val, npad, padi, w,
                                                           int64_t(ox) + int64_t(oy) * pitch1 + int64_t(oz) * pitch2);
                            acc += a * xs[lc + (oz * HY + oy) * HX + ox];
                        }
            }
        }
        const T res = bv - acc;
        if (stop) return;
        r[gi] = res;
        rr = double(res) * double(res);
    }
    if (stop) return;
    if constexpr (NORM) {
        __shared__ double red[256 / kWave];
        for (int off = kWave / 2; off > 0; off >>= 1) rr += __shfl_down(rr, off, kWave);
        if ((threadIdx.x % kWave) == 0) red[threadIdx.x / kWave] = rr;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int k = 0; k < int(blockDim.x / kWave); ++k) s += red[k];
            *part = s;
        }
    }
}

template <int D, int P, class T, bool NORM>
__global__ void __launch_bounds__(256) k_residual(const T *__restrict__ val, int64_t npad, int pitch1, int pitch2,
                                                  int n1, int TX, int TY, int TZ, const T *__restrict__ x,
                                                  const T *__restrict__ b, T *__restrict__ r,
                                                  double *__restrict__ partial, const T *__restrict__ cs, int ulo,
                                                  int uhi, const int *__restrict__ skip,
                                                  const T *__restrict__ kron) {
    extern __shared__ unsigned char smem_raw[];
    int bx = blockIdx.x, by = blockIdx.y;
    if (D == 2) xcd_tile_2d(bx, by);
    double *part = NORM ? partial + (int64_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x : nullptr;
    residual_body<D, P, T, NORM>(val, npad, pitch1, pitch2, n1, TX, TY, TZ, x, b, r, part, cs, ulo, uhi, skip, bx, by,
                                 int(blockIdx.z), reinterpret_cast<T *>(smem_raw), kron);
}

// ------------------------------------------------------------------------
// One colour of the coloured multiplicative Schwarz sweep.  The blocks of the
// colour have centres c with c_k = col_k (mod B) when the colour period equals
// the block width B, so they tile the grid.  Each workgroup owns a tile of
// whole blocks (tile origin shifted by col - hb), reads the colour-start
// iterate x_src over the tile plus a halo of width P, computes the residual
// of every tile point, applies the block inverses and writes x_src + delta
// for every point it owns into x_dst.  Reading x_src and writing x_dst keeps
// all corrections of the colour based on the colour-start iterate.
// For a colour period s > B the same kernel runs with the tile spacing s; the
// points between blocks are copied unchanged.
// The body serves the single-problem kernel and the batched one: tile
// (tbx, tby, tbz) of the colour, smem = LDS of the tile.
template <int D, int P, int B, class T, bool PRE>
__device__ __forceinline__ void colour_body(const T *__restrict__ val, int64_t npad, int pitch1, int pitch2, int n1,
                                            const T *__restrict__ inv, int clsL, int ncls1,
                                            const T *__restrict__ x_src, T *__restrict__ x_dst,
                                            const T *__restrict__ rhs, int x_zero, int ox, int oy, int oz, int S,
                                            int NBX, int NBY, int NBZ, const T *__restrict__ cs, int ulo, int uhi,
                                            const int *__restrict__ skip, const double *__restrict__ r64,
                                            const double *__restrict__ scal, T *__restrict__ rhs_out, int tbx,
                                            int tby, int tbz, unsigned char *smem_raw,
                                            const T *__restrict__ kron = nullptr) {
    // r64 != null (first colour of an FP32 correction sweep, x_zero): the
    // right-hand side is r64 / sigma, cast here and stored to rhs_out for the
    // later colours
    const int stop = skip ? *skip : 0;  // tested before the first store (hides the load latency)
    constexpr int BD = cpow(B, D);
    constexpr int HB = (B - 1) / 2;
    // tile = NBX x NBY (x NBZ) cells of S points; each cell holds one block in
    // its first B x B points
    const int TX = NBX * S, TY = NBY * S, TZ = (D == 3) ? NBZ * S : 1;
    const int HX = TX + 2 * P, HY = TY + 2 * P, HZ = (D == 3) ? TZ + 2 * P : 1;
    T *xs = reinterpret_cast<T *>(smem_raw);
    T *rs = xs + HX * HY * HZ;
    const int gx0 = ox + tbx * TX, gy0 = oy + tby * TY, gz0 = (D == 3) ? oz + tbz * TZ : 0;
    const int nh = HX * HY * HZ;
    // this thread's point, its block and the data it reads from global memory
    // besides the halo: issued first, so that one memory latency covers them
    // and the halo
    const int t = threadIdx.x;
    const int ntile = TX * TY * TZ;
    const int tx = t % TX, ty = (t / TX) % TY, tz = (D == 3) ? t / (TX * TY) : 0;
    const int gx = gx0 + tx, gy = gy0 + ty, gz = gz0 + tz;
    const bool mine = t < ntile && gx >= 0 && gx < n1 && gy >= 0 && gy < n1 && (D == 2 || (gz >= 0 && gz < n1));
    // position inside the cell; points outside the block part are not in any block of this colour
    const int cx = tx % S, cy = ty % S, cz = (D == 3) ? tz % S : 0;
    const bool in_block = cx < B && cy < B && (D == 2 || cz < B);
    const int bx = tx / S, by = ty / S, bz = (D == 3) ? tz / S : 0;
    const int ccx = gx0 + bx * S + HB, ccy = gy0 + by * S + HB, ccz = (D == 3) ? gz0 + bz * S + HB : 0;
    const bool covered = in_block && ccx >= 0 && ccx < n1 && ccy >= 0 && ccy < n1 &&
                         (D == 2 || (ccz >= 0 && ccz < n1));
    const int64_t gi = mine ? (int64_t(gz) * n1 + gy) * n1 + gx : 0;
    T rhs_v = T(0);
    double r64_v = 0.0;
    if (mine && in_block && !r64) rhs_v = rhs[gi];
    if (mine && r64) r64_v = r64[gi];
    // row loc of the block inverse (PRE: held in registers when it is short,
    // for latency-bound launches; batched launches keep the registers free).
    // Not for the 25-entry rows of 2-D 5x5 blocks: held in registers they made
    // the FP32 sweep at p = 5 take 1.6x as long.
    constexpr bool kPreRow = PRE && BD * sizeof(T) <= 128 && !(D == 2 && B == 5);
    constexpr int NR = kPreRow ? BD : 1;
    T irow[NR];
    const T *row = nullptr;
    if (mine && covered) {
        int64_t slot = block_class(ccx, n1, clsL) + int64_t(ncls1) * block_class(ccy, n1, clsL);
        if (D == 3) slot += int64_t(ncls1) * ncls1 * block_class(ccz, n1, clsL);
        const int loc = cx + B * cy + ((D == 3) ? B * B * cz : 0);
        row = inv + (slot * BD + loc) * BD;
        if constexpr (kPreRow) {
#pragma unroll
            for (int l = 0; l < BD; ++l) irow[l] = row[l];
        }
    }
    // one path per wavefront: the interior stencil when all its rows carry it
    // (2-D operators with 1-D factors take every row from the factors)
    const bool uni = cs != nullptr && !(D == 2 && kron != nullptr) &&
                     __all(!mine || point_uniform(gx, gy, gz, ulo, uhi, D));
    // the operator row of a point next to the grid boundary (PRE, 2-D, short
    // rows): loaded with the halo instead of after it
    constexpr int W = cpow(2 * P + 1, D);
    constexpr bool kPreVal = PRE && D == 2 && W * sizeof(T) <= 392;
    T arow[kPreVal ? W : 1];
    if constexpr (kPreVal) {
        if (!uni && !kron && mine && in_block && !x_zero) {
            const int64_t padi = int64_t(gx + P) + int64_t(gy + P) * pitch1;
#pragma unroll
            for (int qy = -P; qy <= P; ++qy)
#pragma unroll
                for (int qx = -P; qx <= P; ++qx) {
                    const int w = (qy + P) * (2 * P + 1) + (qx + P);
                    arow[w] = dia_entry<D, P, T>(val, npad, padi, w, int64_t(qx) + int64_t(qy) * pitch1);
                }
        }
    }
    // the interior stencil (kappa = 1) staged in LDS behind the residuals
    T *css = rs + ntile;
    // 2-D operators that are tensor sums of 1-D factors (kron: rows of Kx, Mx,
    // Ky, My): the x sums of Kx and Mx, once per tile column and window row,
    // behind the stencil; every point then takes its row from 2(2P+1) of them
    T *kxs = css + W, *mxs = kxs + (TY + 2 * P) * TX;
    const bool sf2 = D == 2 && kron != nullptr;
    if (!x_zero) {
        if (cs)
            for (int w = threadIdx.x; w < W; w += blockDim.x) css[w] = cs[w];
        for (int h = threadIdx.x; h < nh; h += blockDim.x) {
            int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
            int hgx = gx0 + hx - P, hgy = gy0 + hy - P, hgz = (D == 3) ? gz0 + hz - P : 0;
            bool in = hgx >= 0 && hgx < n1 && hgy >= 0 && hgy < n1 && (D == 2 || (hgz >= 0 && hgz < n1));
            xs[h] = in ? x_src[(int64_t(hgz) * n1 + hgy) * n1 + hgx] : T(0);
        }
        __syncthreads();
        if constexpr (D == 2) {
            if (sf2) {
                constexpr int W1 = 2 * P + 1;
                const int64_t nw = int64_t(n1) * W1;
                for (int h = threadIdx.x; h < (TY + 2 * P) * TX; h += blockDim.x) {
                    const int c = h % TX, r = h / TX;
                    const int fx = min(max(gx0 + c, 0), n1 - 1);
                    const T *Kx = kron + int64_t(fx) * W1, *Mx = kron + nw + int64_t(fx) * W1;
                    const T *xr = xs + r * HX + c;
                    T kx = T(0), mx = T(0);
#pragma unroll
                    for (int o = 0; o < W1; ++o) {
                        kx += Kx[o] * xr[o];
                        mx += Mx[o] * xr[o];
                    }
                    kxs[h] = kx;
                    mxs[h] = mx;
                }
                __syncthreads();
            }
        }
    }
    const int lc = ((tz + ((D == 3) ? P : 0)) * HY + (ty + P)) * HX + (tx + P);
    T res = T(0);
    T cast_rhs = T(0);
    if (mine) {
        if (r64) cast_rhs = T(r64_v * scal[kScalInvSigma]);
        if (in_block) {
            if (x_zero) {
                res = r64 ? cast_rhs : rhs_v;
            } else {
                const int64_t padi =
                    int64_t(gx + P) + int64_t(gy + P) * pitch1 + ((D == 3) ? int64_t(gz + P) * pitch2 : 0);
                T acc = T(0);
                if (uni && D == 2) {
#pragma unroll
                    for (int qy = -P; qy <= P; ++qy)
#pragma unroll
                        for (int qx = -P; qx <= P; ++qx)
                            acc += css[(qy + P) * (2 * P + 1) + (qx + P)] * xs[lc + qy * HX + qx];
                } else if (uni) {
                    // 3-D: the z loop stays rolled (register budget)
#pragma unroll 1
                    for (int qz = -P; qz <= P; ++qz)
#pragma unroll
                        for (int qy = -P; qy <= P; ++qy)
#pragma unroll
                            for (int qx = -P; qx <= P; ++qx)
                                acc += css[((qz + P) * (2 * P + 1) + (qy + P)) * (2 * P + 1) + (qx + P)] *
                                       xs[lc + (qz * HY + qy) * HX + qx];
                } else if constexpr (D == 2) {
                    if (sf2) {
                        constexpr int W1 = 2 * P + 1;
                        const int64_t nw = int64_t(n1) * W1;
                        const T *Ky = kron + 2 * nw + int64_t(gy) * W1, *My = kron + 3 * nw + int64_t(gy) * W1;
#pragma unroll
                        for (int qy = -P; qy <= P; ++qy) {
                            const int hi = (ty + P + qy) * TX + tx;
                            acc += My[qy + P] * kxs[hi] + Ky[qy + P] * mxs[hi];
                        }
                    } else {
#pragma unroll
                        for (int qy = -P; qy <= P; ++qy)
#pragma unroll
                            for (int qx = -P; qx <= P; ++qx) {
                                const int w = (qy + P) * (2 * P + 1) + (qx + P);
                                T a;
                                if constexpr (kPreVal) a = arow[w];
                                else
                                    a = dia_entry<D, P, T>(val, npad, padi, w, int64_t(qx) + int64_t(qy) * pitch1);
                                acc += a * xs[lc + qy * HX + qx];
                            }
                    }
                } else if (kron) {
                    acc = kron3_row_dot<P, T>(kron, n1, gx, gy, gz, xs, lc, HX, HY);
                } else {
#pragma unroll 1
                    for (int qz = -P; qz <= P; ++qz)
#pragma unroll
                        for (int qy = -P; qy <= P; ++qy)
#pragma unroll
                            for (int qx = -P; qx <= P; ++qx) {
                                const int w = ((qz + P) * (2 * P + 1) + (qy + P)) * (2 * P + 1) + (qx + P);
                                acc += dia_entry<D, P, T>(val, npad, padi, w,
                                                          int64_t(qx) + int64_t(qy) * pitch1 + int64_t(qz) * pitch2) *
                                       xs[lc + (qz * HY + qy) * HX + qx];
                            }
                }
                res = rhs_v - acc;
            }
        }
    }
    if (stop) return;
    if (r64 && mine) rhs_out[gi] = cast_rhs;
    if (t < ntile) rs[t] = res;
    __syncthreads();
    if (!mine) return;
    T xi = x_zero ? T(0) : xs[lc];
    T delta = T(0);
    if (covered) {
        const int base = ((bz * S) * TY + by * S) * TX + bx * S;
#pragma unroll
        for (int l = 0; l < BD; ++l) {
            const int lx = l % B, ly = (l / B) % B, lz = (D == 3) ? l / (B * B) : 0;
            T a;
            if constexpr (kPreRow) a = irow[l];
            else a = row[l];
            delta += a * rs[base + (lz * TY + ly) * TX + lx];
        }
    }
    x_dst[gi] = xi + delta;
}

// PRE: operands held in registers ahead of use (latency-bound grids)
template <int D, int P, int B, class T, bool PRE>
__global__ void __launch_bounds__(kColourThreads) k_colour(const T *__restrict__ val, int64_t npad, int pitch1, int pitch2,
                                                 int n1, const T *__restrict__ inv, int clsL, int ncls1, const T *__restrict__ x_src, T *__restrict__ x_dst,
                                                 const T *__restrict__ rhs, int x_zero, int ox, int oy, int oz,
                                                 int S, int NBX, int NBY, int NBZ, const T *__restrict__ cs, int ulo,
                                                 int uhi, const int *__restrict__ skip,
                                                 const double *__restrict__ r64, const double *__restrict__ scal,
                                                 T *__restrict__ rhs_out, const T *__restrict__ kron) {
    extern __shared__ unsigned char smem_raw[];
    int bx = blockIdx.x, by = blockIdx.y;
    if (D == 2) xcd_tile_2d(bx, by);
    colour_body<D, P, B, T, PRE>(val, npad, pitch1, pitch2, n1, inv, clsL, ncls1, x_src, x_dst, rhs, x_zero, ox, oy,
                                  oz, S, NBX, NBY, NBZ, cs, ulo, uhi, skip, r64, scal, rhs_out, bx, by,
                                  int(blockIdx.z), smem_raw, kron);
}

// ------------------------------------------------------------------------
// One step of the lexicographic Schwarz sweep: every block of the step (they
// do not interact) computes its residual from u, applies its inverse and
// updates u in place.  One workgroup per block, one thread per block point.
template <int D, int P, int B>
__global__ void __launch_bounds__(128) k_lex_step(const double *__restrict__ val, int64_t npad, int pitch1,
                                                  int pitch2, int n1, const double *__restrict__ inv,
                                                  const int *__restrict__ cls, int ncls1,
                                                  const int *__restrict__ blocks, int first, double *u,
                                                  const double *__restrict__ b, const int *__restrict__ skip) {
    if (skip && *skip) return;
    constexpr int BD = cpow(B, D);
    constexpr int HB = (B - 1) / 2;
    __shared__ double rs[BD];
    const int j = blocks[first + blockIdx.x];
    const int jx = j % n1, jy = (j / n1) % n1, jz = (D == 3) ? j / (n1 * n1) : 0;
    const int l = threadIdx.x;
    int gx = 0, gy = 0, gz = 0;
    bool in = false;
    if (l < BD) {
        gx = jx + l % B - HB;
        gy = jy + (l / B) % B - HB;
        gz = (D == 3) ? jz + l / (B * B) - HB : 0;
        in = gx >= 0 && gx < n1 && gy >= 0 && gy < n1 && (D == 2 || (gz >= 0 && gz < n1));
        double r = 0.0;
        if (in) {
            const int64_t gi = (int64_t(gz) * n1 + gy) * n1 + gx;
            const int64_t padi = int64_t(gx + P) + int64_t(gy + P) * pitch1 + ((D == 3) ? int64_t(gz + P) * pitch2 : 0);
            double acc = 0.0;
            for (int qz = ((D == 3) ? -P : 0); qz <= ((D == 3) ? P : 0); ++qz)
                for (int qy = -P; qy <= P; ++qy)
                    for (int qx = -P; qx <= P; ++qx) {
                        const int hx = gx + qx, hy = gy + qy, hz = gz + qz;
                        if (hx < 0 || hx >= n1 || hy < 0 || hy >= n1 || (D == 3 && (hz < 0 || hz >= n1))) continue;
                        const int w = ((D == 3) ? (qz + P) * (2 * P + 1) * (2 * P + 1) : 0) + (qy + P) * (2 * P + 1) + (qx + P);
                        acc += dia_entry<D, P, double>(val, npad, padi, w,
                                                       int64_t(qx) + int64_t(qy) * pitch1 + int64_t(qz) * pitch2) *
                               u[(int64_t(hz) * n1 + hy) * n1 + hx];
                    }
            r = b[gi] - acc;
        }
        rs[l] = r;
    }
    __syncthreads();
    if (l < BD && in) {
        int64_t slot = cls[jx] + int64_t(ncls1) * cls[jy];
        if (D == 3) slot += int64_t(ncls1) * ncls1 * cls[jz];
        const double *row = inv + (slot * BD + l) * BD;
        double delta = 0.0;
        for (int k = 0; k < BD; ++k) delta += row[k] * rs[k];
        u[(int64_t(gz) * n1 + gy) * n1 + gx] += delta;
    }
}

// ------------------------------------------------------------------------
// The whole lexicographic sweep in one workgroup (small grids): the iterate,
// the right-hand side and the step schedule live in LDS, the steps run one
// after the other with a barrier between them, each step's blocks in
// parallel, one thread per block point.  A thread loads its inverse row and,
// next to the grid boundary, its operator row (2-D, p <= 3) one step ahead,
// so the memory latency overlaps the previous step instead of adding to it.
// Same arithmetic as k_lex_step (interior rows read the interior stencil,
// which equals their diagonals bit for bit; out-of-grid neighbours are
// skipped), so the result equals the step-by-step launches.
constexpr int kLexThreads = 256;

// one thread's point in one step and the operands it loads for it
template <int D, int P, int B>
struct LexPoint {
    static constexpr int BD = cpow(B, D);
    static constexpr bool kPreA = D == 2 && P <= 3;  // operator row held in registers
    static constexpr int NA = kPreA ? cpow(2 * P + 1, D) : 1;
    bool act = false, in = false, uni = false;
    int gx = 0, gy = 0, gz = 0, gi = 0;
    double row[BD];
    double a[NA];
};

template <int D, int P, int B>
__device__ __forceinline__ void lex_point_load(LexPoint<D, P, B> &q, int st, int nsteps, const int *off,
                                               const int *blk, int n1, const double *__restrict__ val,
                                               int64_t npad, int pitch1, const double *__restrict__ inv, int clsL,
                                               int ncls1, bool has_cs, int ulo, int uhi) {
    constexpr int BD = cpow(B, D);
    constexpr int HB = (B - 1) / 2;
    const int idx = threadIdx.x, l = idx % BD;
    q.act = false;
    q.in = false;
    if (st >= nsteps) return;
    const int first = off[st], cnt = off[st + 1] - first;
    q.act = idx < cnt * BD;
    if (!q.act) return;
    const int j = blk[first + idx / BD];
    const int jx = j % n1, jy = (j / n1) % n1, jz = (D == 3) ? j / (n1 * n1) : 0;
    q.gx = jx + l % B - HB;
    q.gy = jy + (l / B) % B - HB;
    q.gz = (D == 3) ? jz + l / (B * B) - HB : 0;
    q.in = q.gx >= 0 && q.gx < n1 && q.gy >= 0 && q.gy < n1 && (D == 2 || (q.gz >= 0 && q.gz < n1));
    if (!q.in) return;
    q.gi = (q.gz * n1 + q.gy) * n1 + q.gx;
    q.uni = has_cs && point_uniform(q.gx, q.gy, q.gz, ulo, uhi, D);
    int64_t slot = block_class(jx, n1, clsL) + int64_t(ncls1) * block_class(jy, n1, clsL);
    if (D == 3) slot += int64_t(ncls1) * ncls1 * block_class(jz, n1, clsL);
    const double *ir = inv + (slot * BD + l) * BD;
#pragma unroll
    for (int k = 0; k < BD; ++k) q.row[k] = ir[k];
    if constexpr (LexPoint<D, P, B>::kPreA) {
        if (!q.uni) {
            const int64_t padi = int64_t(q.gx + P) + int64_t(q.gy + P) * pitch1;
#pragma unroll
            for (int qy = -P; qy <= P; ++qy)
#pragma unroll
                for (int qx = -P; qx <= P; ++qx) {
                    const int hx = q.gx + qx, hy = q.gy + qy;
                    const bool ok = hx >= 0 && hx < n1 && hy >= 0 && hy < n1;
                    const int w = (qy + P) * (2 * P + 1) + (qx + P);
                    q.a[w] = ok ? dia_entry<D, P, double>(val, npad, padi, w, int64_t(qx) + int64_t(qy) * pitch1)
                                : 0.0;
                }
        }
    }
}

template <int D, int P, int B>
__global__ void __launch_bounds__(kLexThreads) k_lex_sweep(const double *__restrict__ val, int64_t npad, int pitch1,
                                                           int pitch2, int n1, const double *__restrict__ inv,
                                                           int clsL, int ncls1, const int *__restrict__ blocks,
                                                           const int *__restrict__ offs, int nsteps, double *u,
                                                           const double *__restrict__ b,
                                                           const double *__restrict__ cs, int ulo, int uhi,
                                                           const int *__restrict__ skip) {
    if (skip && *skip) return;
    constexpr int BD = cpow(B, D);
    constexpr int W = cpow(2 * P + 1, D);
    constexpr int WP = cpow(2 * P + 1, 2);  // one z plane of the stencil
    using LP = LexPoint<D, P, B>;
    extern __shared__ unsigned char smem_raw[];
    const int n = (D == 3) ? n1 * n1 * n1 : n1 * n1;
    double *us = reinterpret_cast<double *>(smem_raw);
    double *bs = us + n;
    double *css = bs + n;
    double *rs = css + W;                                           // one step's block residuals
    int *blk = reinterpret_cast<int *>(rs + kLexThreads);           // the schedule
    int *off = blk + n;                                             // step offsets
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        us[i] = u[i];
        bs[i] = b[i];
        blk[i] = blocks[i];
    }
    for (int i = threadIdx.x; i <= nsteps; i += blockDim.x) off[i] = offs[i];
    if (cs)
        for (int w = threadIdx.x; w < W; w += blockDim.x) css[w] = cs[w];
    __syncthreads();
    const int idx = threadIdx.x;
    LP cur, nxt;
    lex_point_load<D, P, B>(cur, 0, nsteps, off, blk, n1, val, npad, pitch1, inv, clsL, ncls1, cs != nullptr, ulo,
                            uhi);
    for (int st = 0; st < nsteps; ++st) {
        // the next step's operands: in flight during this step
        lex_point_load<D, P, B>(nxt, st + 1, nsteps, off, blk, n1, val, npad, pitch1, inv, clsL, ncls1,
                                cs != nullptr, ulo, uhi);
        if (cur.act) {
            double r = 0.0;
            if (cur.in) {
                const int gx = cur.gx, gy = cur.gy, gz = cur.gz, gi = cur.gi;
                double acc = 0.0;
                if (cur.uni) {
                    // every neighbour lies inside the grid
#pragma unroll 1
                    for (int qz = ((D == 3) ? -P : 0); qz <= ((D == 3) ? P : 0); ++qz)
#pragma unroll
                        for (int qy = -P; qy <= P; ++qy)
#pragma unroll
                            for (int qx = -P; qx <= P; ++qx)
                                acc += css[(D == 3 ? (qz + P) * WP : 0) + (qy + P) * (2 * P + 1) + (qx + P)] *
                                       us[gi + (qz * n1 + qy) * n1 + qx];
                } else if constexpr (LP::kPreA) {
#pragma unroll
                    for (int qy = -P; qy <= P; ++qy)
#pragma unroll
                        for (int qx = -P; qx <= P; ++qx) {
                            const int hx = gx + qx, hy = gy + qy;
                            const bool ok = hx >= 0 && hx < n1 && hy >= 0 && hy < n1;
                            if (ok) acc += cur.a[(qy + P) * (2 * P + 1) + (qx + P)] * us[gi + qy * n1 + qx];
                        }
                } else {
                    const int64_t padi =
                        int64_t(gx + P) + int64_t(gy + P) * pitch1 + ((D == 3) ? int64_t(gz + P) * pitch2 : 0);
                    // operator entries fetched RY stencil rows at a time (all of a
                    // z plane for p <= 3), then accumulated in the skip order
                    constexpr int RY = (P <= 3) ? 2 * P + 1 : 1;
#pragma unroll 1
                    for (int qz = ((D == 3) ? -P : 0); qz <= ((D == 3) ? P : 0); ++qz) {
                        const bool zok = D == 2 || (gz + qz >= 0 && gz + qz < n1);
#pragma unroll 1
                        for (int qy0 = -P; qy0 <= P; qy0 += RY) {
                            double a[RY * (2 * P + 1)];
#pragma unroll
                            for (int ry = 0; ry < RY; ++ry)
#pragma unroll
                                for (int qx = -P; qx <= P; ++qx) {
                                    const int qy = qy0 + ry, hx = gx + qx, hy = gy + qy;
                                    const bool ok = zok && hx >= 0 && hx < n1 && hy >= 0 && hy < n1;
                                    const int w = (D == 3 ? (qz + P) * WP : 0) + (qy + P) * (2 * P + 1) + (qx + P);
                                    a[ry * (2 * P + 1) + (qx + P)] =
                                        ok ? dia_entry<D, P, double>(val, npad, padi, w,
                                                                     int64_t(qx) + int64_t(qy) * pitch1 +
                                                                         int64_t(qz) * pitch2)
                                           : 0.0;
                                }
#pragma unroll
                            for (int ry = 0; ry < RY; ++ry)
#pragma unroll
                                for (int qx = -P; qx <= P; ++qx) {
                                    const int qy = qy0 + ry, hx = gx + qx, hy = gy + qy;
                                    const bool ok = zok && hx >= 0 && hx < n1 && hy >= 0 && hy < n1;
                                    if (ok) acc += a[ry * (2 * P + 1) + (qx + P)] * us[gi + (qz * n1 + qy) * n1 + qx];
                                }
                        }
                    }
                }
                r = bs[gi] - acc;
            }
            rs[idx] = r;
        }
        __syncthreads();
        if (cur.act && cur.in) {
            const double *rb = rs + (idx / BD) * BD;
            double delta = 0.0;
#pragma unroll
            for (int k = 0; k < BD; ++k) delta += cur.row[k] * rb[k];
            us[cur.gi] += delta;
        }
        __syncthreads();
        cur = nxt;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) u[i] = us[i];
}

// ------------------------------------------------------------------------
// Inverse of every block matrix A^{B_j} = V_j A V_j^T (one per slot) by
// in-place Gauss-Jordan elimination without pivoting (the block matrices are
// symmetric positive definite).  Block members outside the grid get identity
// rows/columns during the elimination and zero rows/columns in the result.
template <int D, int B>
__global__ void __launch_bounds__(kWave) k_block_inverse(const double *__restrict__ val, int64_t npad, int pitch1,
                                                         int pitch2, int n1, int P, const int64_t *__restrict__ reps,
                                                         double *__restrict__ inv, int *__restrict__ err) {
    constexpr int BD = cpow(B, D);
    constexpr int HB = (B - 1) / 2;
    __shared__ double a[BD * BD];
    __shared__ double col[BD];
    __shared__ int member_in[BD];
    __shared__ int64_t member_pad[BD];
    __shared__ int mx[BD], my[BD], mz[BD];
    const int64_t j = reps[blockIdx.x];
    const int jx = int(j % n1), jy = int((j / n1) % n1), jz = (D == 3) ? int(j / (int64_t(n1) * n1)) : 0;
    const int W1 = 2 * P + 1;
    const int W = (D == 3) ? W1 * W1 * W1 : W1 * W1;
    const int c0 = (W - 1) / 2;
    for (int l = threadIdx.x; l < BD; l += blockDim.x) {
        int gx = jx + l % B - HB, gy = jy + (l / B) % B - HB, gz = (D == 3) ? jz + l / (B * B) - HB : 0;
        mx[l] = gx;
        my[l] = gy;
        mz[l] = gz;
        member_in[l] = gx >= 0 && gx < n1 && gy >= 0 && gy < n1 && (D == 2 || (gz >= 0 && gz < n1));
        member_pad[l] = int64_t(gx + P) + int64_t(gy + P) * pitch1 + ((D == 3) ? int64_t(gz + P) * pitch2 : 0);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < BD * BD; e += blockDim.x) {
        const int r = e / BD, c = e % BD;
        double v = (r == c) ? 1.0 : 0.0;
        if (member_in[r] && member_in[c]) {
            const int qx = mx[c] - mx[r], qy = my[c] - my[r], qz = mz[c] - mz[r];
            if (qx >= -P && qx <= P && qy >= -P && qy <= P && qz >= -P && qz <= P) {
                const int w = ((D == 3) ? (qz + P) * W1 * W1 : 0) + (qy + P) * W1 + (qx + P);
                if (w >= c0) v = val[int64_t(w - c0) * npad + member_pad[r]];
                else v = val[int64_t(c0 - w) * npad + member_pad[c]];
            } else {
                v = 0.0;
            }
        }
        a[e] = v;
    }
    __syncthreads();
    for (int k = 0; k < BD; ++k) {
        const double piv = a[k * BD + k];
        if (threadIdx.x == 0 && !(piv > 0.0)) atomicOr(err, 1);
        for (int i = threadIdx.x; i < BD; i += blockDim.x) col[i] = a[i * BD + k];
        __syncthreads();
        for (int c = threadIdx.x; c < BD; c += blockDim.x) a[k * BD + c] = ((c == k) ? 1.0 : a[k * BD + c]) / piv;
        __syncthreads();
        for (int e = threadIdx.x; e < BD * BD; e += blockDim.x) {
            const int r = e / BD, c = e % BD;
            if (r == k) continue;
            a[e] = ((c == k) ? 0.0 : a[e]) - col[r] * a[k * BD + c];
        }
        __syncthreads();
    }
    double *out = inv + int64_t(blockIdx.x) * BD * BD;
    for (int e = threadIdx.x; e < BD * BD; e += blockDim.x) {
        const int r = e / BD, c = e % BD;
        out[e] = (member_in[r] && member_in[c]) ? a[e] : 0.0;
    }
}

// ------------------------------------------------------------------------
// Fixed-order reduction of the per-workgroup partial sums into ||r||_2 and
// the scaling used by the FP32 correction cycle.  book != nullptr: the
// device-side convergence test after a cycle (record the relative residual,
// count the cycle, raise the stop flag).
__device__ __forceinline__ void finalize_body(const double *__restrict__ partial, int np, double *scal,
                                              int scale_fp32, int *book, double *hist, int hist_cap) {
    if (book && book[kFlagDone]) return;
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nrm = sqrt(red[0]);
        const double sigma = (scale_fp32 && nrm > 0.0) ? nrm : 1.0;
        scal[kScalNorm] = nrm;
        scal[kScalSigma] = sigma;
        scal[kScalInvSigma] = 1.0 / sigma;
        if (book) {
            const double r0 = scal[kScalR0];
            const double rel = r0 > 0.0 ? nrm / r0 : 0.0;
            const int k = book[kFlagIter];
            if (k < hist_cap) hist[k] = rel;
            book[kFlagIter] = k + 1;
            int status = 0;
            if (!isfinite(rel) || rel > 1e3) status = 2;
            else if (rel > scal[kScalTol] && k + 1 >= int(scal[kScalMaxCycles])) status = 1;
            book[kFlagStatus] = status;
            book[kFlagDone] = (status != 0 || rel <= scal[kScalTol]) ? 1 : 0;
        }
    }
}

__global__ void __launch_bounds__(256) k_norm_finalize(const double *__restrict__ partial, int np, double *scal,
                                                       int scale_fp32, int *book, double *hist, int hist_cap) {
    finalize_body(partial, np, scal, scale_fp32, book, hist, hist_cap);
}

// Start of a solve: the norm just computed is r0; set the stopping data.
__device__ __forceinline__ void init_body(double *scal, int *flags, double tol, int max_cycles) {
    const double r0 = scal[kScalNorm];
    scal[kScalR0] = r0;
    scal[kScalTol] = tol;
    scal[kScalMaxCycles] = double(max_cycles);
    int status = 0, done = 0;
    if (!isfinite(r0)) {
        status = 2;
        done = 1;
    } else if (r0 == 0.0 || tol >= 1.0) {
        done = 1;
    } else if (max_cycles == 0) {
        status = 1;
        done = 1;
    }
    flags[kFlagDone] = done;
    flags[kFlagIter] = 0;
    flags[kFlagStatus] = status;
}

__global__ void k_solve_init(double *scal, int *flags, double tol, int max_cycles) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    init_body(scal, flags, tol, max_cycles);
}

template <class T>
__global__ void k_cast_scale(const double *__restrict__ r64, T *__restrict__ out, const double *__restrict__ scal,
                             int64_t n, const int *__restrict__ skip) {
    const int stop = skip ? *skip : 0;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T v = T(r64[i] * scal[kScalInvSigma]);
    if (stop) return;
    out[i] = v;
}

// ------------------------------------------------------------ dispatch --
template <int D, int P>
struct TileShape;
template <int P>
struct TileShape<2, P> {
    static constexpr int TX = 64, TY = 4, TZ = 1;
};
template <int P>
struct TileShape<3, P> {
    static constexpr int TX = 16, TY = 8, TZ = 2;
};

// 1-D factors for the 3-D boundary rows (null: read the diagonals)
template <class T>
const T *kron_factors(const Problem &Pb) {
    // 2-D: the direction-dependent factor rows of the annulus (null otherwise)
    if (Pb.dim == 2)
        return std::is_same<T, double>::value ? reinterpret_cast<const T *>(Pb.fac2d64.ptr)
                                              : reinterpret_cast<const T *>(Pb.fac2d32.ptr);
    return std::is_same<T, double>::value ? reinterpret_cast<const T *>(Pb.kron64.ptr)
                                          : reinterpret_cast<const T *>(Pb.kron32.ptr);
}

template <class T>
const T *uniform_stencil(const Problem &Pb) {
    return std::is_same<T, double>::value ? reinterpret_cast<const T *>(Pb.cs64.ptr)
                                          : reinterpret_cast<const T *>(Pb.cs32.ptr);
}

template <int D, int P, class T, bool NORM>
void residual_launch(const Problem &Pb, const T *val, const T *x, const T *b, T *r, double *partial, int &nblocks,
                     bool scale_fp32, bool book, hipStream_t s) {
    // column-blocked 2-D kernel on large grids (bandwidth regime); the small-tile
    // kernel below keeps more workgroups in flight on small ones
    if constexpr (D == 2) if (Pb.fine.n >= (int64_t(1) << 20)) {
        launch_residual2d<T>(Pb, val, x, b, r, NORM ? partial : nullptr, s);
        nblocks = int(residual2d_workgroups(Pb));
        if (NORM)
            hipLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(256), 0, s, Pb.partial.as<double>(), nblocks,
                               Pb.scal.as<double>(), scale_fp32 ? 1 : 0, book ? dev_flags(Pb) : nullptr,
                               dev_hist(Pb), Pb.hist_cap);
        return;
    }
    if constexpr (D == 3) if (residual3d_sf_ok(Pb)) {
        // kappa = 1: sum factorisation over the 1-D factors
        launch_residual3d_sf<T, NORM>(Pb, x, b, r, NORM ? partial : nullptr, s);
        nblocks = int(residual3d_sf_workgroups(Pb));
        if (NORM)
            hipLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(256), 0, s, Pb.partial.as<double>(), nblocks,
                               Pb.scal.as<double>(), scale_fp32 ? 1 : 0, book ? dev_flags(Pb) : nullptr,
                               dev_hist(Pb), Pb.hist_cap);
        return;
    }
    using TS = TileShape<D, P>;
    const int n1 = Pb.fine.n1;
    dim3 grid((n1 + TS::TX - 1) / TS::TX, (n1 + TS::TY - 1) / TS::TY, D == 3 ? (n1 + TS::TZ - 1) / TS::TZ : 1);
    const size_t shm = (size_t(TS::TX + 2 * P) * (TS::TY + 2 * P) * (D == 3 ? TS::TZ + 2 * P : 1) +
                        size_t(cpow(2 * P + 1, D))) * sizeof(T);
    nblocks = int(grid.x * grid.y * grid.z);
    hipLaunchKernelGGL((k_residual<D, P, T, NORM>), grid, dim3(TS::TX * TS::TY * TS::TZ), shm, s, val, Pb.A.npad,
                       Pb.A.pitch[1], Pb.A.pitch[2], n1, TS::TX, TS::TY, TS::TZ, x, b, r, partial,
                       uniform_stencil<T>(Pb), Pb.ulo, Pb.uhi, Pb.skip,
                       (D == 2) ? static_cast<const T *>(colour_factor_rows(Pb, std::is_same<T, double>::value))
                                : kron_factors<T>(Pb));
    if (NORM)
        hipLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(256), 0, s, Pb.partial.as<double>(), nblocks,
                           Pb.scal.as<double>(), scale_fp32 ? 1 : 0, book ? dev_flags(Pb) : nullptr, dev_hist(Pb),
                           Pb.hist_cap);
}

#define IGA2L_DISPATCH_P2(F, ...)                                   \
    switch (Pb.p) {                                                 \
        case 1: F<2, 1>(__VA_ARGS__); break;                        \
        case 2: F<2, 2>(__VA_ARGS__); break;                        \
        case 3: F<2, 3>(__VA_ARGS__); break;                        \
        case 4: F<2, 4>(__VA_ARGS__); break;                        \
        case 5: F<2, 5>(__VA_ARGS__); break;                        \
        case 6: F<2, 6>(__VA_ARGS__); break;                        \
        case 7: F<2, 7>(__VA_ARGS__); break;                        \
        case 8: F<2, 8>(__VA_ARGS__); break;                        \
        default: throw Error{IGA2L_EUNSUPPORTED, "degree out of range"}; \
    }
#define IGA2L_DISPATCH_P3(F, ...)                                   \
    switch (Pb.p) {                                                 \
        case 1: F<3, 1>(__VA_ARGS__); break;                        \
        case 2: F<3, 2>(__VA_ARGS__); break;                        \
        case 3: F<3, 3>(__VA_ARGS__); break;                        \
        case 4: F<3, 4>(__VA_ARGS__); break;                        \
        default: throw Error{IGA2L_EUNSUPPORTED, "3-D degree out of range"}; \
    }

template <int D, int P>
void res64_dp(const Problem &Pb, const double *u, const double *b, double *r, bool norm, bool scale_fp32,
              bool book, hipStream_t s) {
    int nb = 0;
    if (norm) {
        IGA2L_REQUIRE(residual_workgroups(Pb) <= Pb.npartial, IGA2L_EUNSUPPORTED,
                      "grid too large for the norm workspace");
        residual_launch<D, P, double, true>(Pb, Pb.A.v64.as<double>(), u, b, r, Pb.partial.as<double>(), nb,
                                            scale_fp32, book, s);
    } else {
        residual_launch<D, P, double, false>(Pb, Pb.A.v64.as<double>(), u, b, r, nullptr, nb, false, false, s);
    }
}

template <int D, int P, class T>
void defect_dp(const Problem &Pb, const T *e, const T *rhs, T *d, hipStream_t s) {
    int nb = 0;
    const T *val = std::is_same<T, double>::value ? reinterpret_cast<const T *>(Pb.A.v64.ptr)
                                                  : reinterpret_cast<const T *>(Pb.A.v32.ptr);
    residual_launch<D, P, T, false>(Pb, val, e, rhs, d, nullptr, nb, false, false, s);
}

template <int D, int P, int B, class T>
void colour_launch(const Problem &Pb, int cx, int cy, int cz, int S, const T *x_src, T *x_dst, const T *rhs,
                   bool x_zero, const double *r64, T *rhs_out, hipStream_t s, int tile_nbx = 0, int tile_nby = 0) {
    // 2-D kappa = 1 on large grids, colour period b: streamed (explicit tile
    // shapes ask for this kernel)
    if constexpr (D == 2)
        if (tile_nbx == 0 && tile_nby == 0 &&
            colour2d_stream(Pb, cx, cy, S, x_src, x_dst, rhs, x_zero, r64, rhs_out, std::is_same<T, double>::value, s))
            return;
    if constexpr (D == 3 && B == 3) if (colour3d_sf_ok(Pb, S)) {
        // kappa = 1, colour period 3: sum-factorised residual, shared inverse on MFMA
        launch_colour3d_sf<T>(Pb, cx, cy, cz, x_src, x_dst, rhs, x_zero, r64, rhs_out, s);
        return;
    }
    const int n1 = Pb.fine.n1;
    constexpr int HB = (B - 1) / 2;
    constexpr int pr = std::is_same<T, double>::value ? 0 : 1;
    int nbx = tile_nbx >= 1 ? tile_nbx : Pb.tile_bx[pr], nby = tile_nby >= 1 ? tile_nby : Pb.tile_by[pr];
    int nbz = (D == 3) ? Pb.tile_bz : 1;
    // keep the tile within one workgroup of at most kColourThreads threads
    while (nbx * S * nby * S * ((D == 3) ? nbz * S : 1) > kColourThreads) {
        if (nby > 1) --nby;
        else if (nbx > 1) --nbx;
        else if (nbz > 1) --nbz;
        else break;
    }
    const int TX = nbx * S, TY = nby * S, TZ = (D == 3) ? nbz * S : 1;
    IGA2L_REQUIRE(TX * TY * TZ <= kColourThreads, IGA2L_EUNSUPPORTED, "colour period too large for one workgroup");
    // tile origins: aligned with the colour's blocks and at or before index 0
    int ox = cx - HB, oy = cy - HB, oz = (D == 3) ? cz - HB : 0;
    if (ox > 0) ox -= S;
    if (oy > 0) oy -= S;
    if (oz > 0) oz -= S;
    dim3 grid((n1 - ox + TX - 1) / TX, (n1 - oy + TY - 1) / TY, D == 3 ? (n1 - oz + TZ - 1) / TZ : 1);
    const int threads = ((TX * TY * TZ + kWave - 1) / kWave) * kWave;
    const T *fac2 = (D == 2) ? static_cast<const T *>(colour_factor_rows(Pb, std::is_same<T, double>::value))
                             : kron_factors<T>(Pb);
    const size_t sf2_lds = (D == 2 && fac2) ? 2 * size_t(TY + 2 * Pb.p) * TX : 0;
    const size_t shm = (size_t(TX + 2 * Pb.p) * (TY + 2 * Pb.p) * (D == 3 ? TZ + 2 * Pb.p : 1) + size_t(TX) * TY * TZ +
                        size_t(cpow(2 * P + 1, D)) + sf2_lds) *
                       sizeof(T);
    const T *val = std::is_same<T, double>::value ? reinterpret_cast<const T *>(Pb.A.v64.ptr)
                                                  : reinterpret_cast<const T *>(Pb.A.v32.ptr);
    const T *inv = std::is_same<T, double>::value ? reinterpret_cast<const T *>(Pb.Inv64.ptr)
                                                  : reinterpret_cast<const T *>(Pb.Inv32.ptr);
    // small grids are latency-bound: operands in registers ahead of use; large
    // ones keep the registers for occupancy
    auto kern = Pb.fine.n < kColourPreMaxN ? k_colour<D, P, B, T, true> : k_colour<D, P, B, T, false>;
    hipLaunchKernelGGL(kern, grid, dim3(threads), shm, s, val, Pb.A.npad, Pb.A.pitch[1],
                       Pb.A.pitch[2], n1, inv, class_split(Pb), Pb.ncls1, x_src, x_dst, rhs, x_zero ? 1 : 0, ox,
                       oy, oz, S, nbx, nby, nbz, uniform_stencil<T>(Pb), Pb.ulo, Pb.uhi, Pb.skip, r64,
                       Pb.scal.as<double>(), rhs_out, fac2);
}

template <int D, int P, class T>
void colour_dp(const Problem &Pb, int cx, int cy, int cz, int S, const T *x_src, T *x_dst, const T *rhs, bool x_zero,
               const double *r64, T *rhs_out, hipStream_t s, int nbx = 0, int nby = 0) {
    switch (Pb.bw) {
        case 1: colour_launch<D, P, 1, T>(Pb, cx, cy, cz, S, x_src, x_dst, rhs, x_zero, r64, rhs_out, s, nbx, nby); break;
        case 3: colour_launch<D, P, 3, T>(Pb, cx, cy, cz, S, x_src, x_dst, rhs, x_zero, r64, rhs_out, s, nbx, nby); break;
        case 5:
            if constexpr (D == 2)
                colour_launch<D, P, 5, T>(Pb, cx, cy, cz, S, x_src, x_dst, rhs, x_zero, r64, rhs_out, s, nbx, nby);
            else throw Error{IGA2L_EUNSUPPORTED, "3-D block width must be 1 or 3"};
            break;
        case 7:
            if constexpr (D == 2)
                colour_launch<D, P, 7, T>(Pb, cx, cy, cz, S, x_src, x_dst, rhs, x_zero, r64, rhs_out, s, nbx, nby);
            else throw Error{IGA2L_EUNSUPPORTED, "3-D block width must be 1 or 3"};
            break;
        default: throw Error{IGA2L_EUNSUPPORTED, "block width must be 1, 3, 5 or 7"};
    }
}

template <int D, int P, int B>
void lex_launch(const Problem &Pb, int step, double *u, const double *b, hipStream_t s) {
    const int first = Pb.lex_off[step], cnt = Pb.lex_off[step + 1] - first;
    constexpr int BD = cpow(B, D);
    const int threads = BD <= 64 ? 64 : 128;
    hipLaunchKernelGGL((k_lex_step<D, P, B>), dim3(cnt), dim3(threads), 0, s, Pb.A.v64.as<double>(), Pb.A.npad,
                       Pb.A.pitch[1], Pb.A.pitch[2], Pb.fine.n1, Pb.Inv64.as<double>(), Pb.cls_d.as<int>(), Pb.ncls1,
                       Pb.lex_blocks.as<int>(), first, u, b, Pb.skip);
}

// iterate, right-hand side, interior stencil, one step's block residuals,
// schedule and step offsets
size_t lex_sweep_lds(const Problem &Pb) {
    const int64_t w = (Pb.dim == 3) ? int64_t(2 * Pb.p + 1) * (2 * Pb.p + 1) * (2 * Pb.p + 1)
                                    : int64_t(2 * Pb.p + 1) * (2 * Pb.p + 1);
    return size_t(2 * Pb.fine.n + w + kLexThreads) * sizeof(double) +
           size_t(Pb.fine.n + int64_t(Pb.lex_off.size())) * sizeof(int);
}

template <int D, int P, int B>
void lex_sweep_launch(const Problem &Pb, double *u, const double *b, hipStream_t s) {
    const size_t shm = lex_sweep_lds(Pb);
    const int nsteps = int(Pb.lex_off.size()) - 1;
    hipLaunchKernelGGL((k_lex_sweep<D, P, B>), dim3(1), dim3(kLexThreads), shm, s, Pb.A.v64.as<double>(), Pb.A.npad,
                       Pb.A.pitch[1], Pb.A.pitch[2], Pb.fine.n1, Pb.Inv64.as<double>(), class_split(Pb), Pb.ncls1,
                       Pb.lex_blocks.as<int>(), Pb.lex_off_d.as<int>(), nsteps, u, b, uniform_stencil<double>(Pb),
                       Pb.ulo, Pb.uhi, Pb.skip);
}

template <int D, int P>
void lex_sweep_dp(const Problem &Pb, double *u, const double *b, hipStream_t s) {
    switch (Pb.bw) {
        case 1: lex_sweep_launch<D, P, 1>(Pb, u, b, s); break;
        case 3: lex_sweep_launch<D, P, 3>(Pb, u, b, s); break;
        case 5:
            if constexpr (D == 2) lex_sweep_launch<D, P, 5>(Pb, u, b, s);
            else throw Error{IGA2L_EUNSUPPORTED, "3-D block width must be 1 or 3"};
            break;
        case 7:
            if constexpr (D == 2) lex_sweep_launch<D, P, 7>(Pb, u, b, s);
            else throw Error{IGA2L_EUNSUPPORTED, "3-D block width must be 1 or 3"};
            break;
        default: throw Error{IGA2L_EUNSUPPORTED, "block width must be 1, 3, 5 or 7"};
    }
}

template <int D, int P>
void lex_dp(const Problem &Pb, int step, double *u, const double *b, hipStream_t s) {
    switch (Pb.bw) {
        case 1: lex_launch<D, P, 1>(Pb, step, u, b, s); break;
        case 3: lex_launch<D, P, 3>(Pb, step, u, b, s); break;
        case 5:
            if constexpr (D == 2) lex_launch<D, P, 5>(Pb, step, u, b, s);
            else throw Error{IGA2L_EUNSUPPORTED, "3-D block width must be 1 or 3"};
            break;
        case 7:
            if constexpr (D == 2) lex_launch<D, P, 7>(Pb, step, u, b, s);
            else throw Error{IGA2L_EUNSUPPORTED, "3-D block width must be 1 or 3"};
            break;
        default: throw Error{IGA2L_EUNSUPPORTED, "block width must be 1, 3, 5 or 7"};
    }
}

// ----------------------------------------------------------- batched --
template <class T>
constexpr int prec_slot() { return std::is_same<T, double>::value ? 0 : 1; }

template <int P, class T, bool NORM>
__global__ void __launch_bounds__(256) kb_residual(const BatchProb *__restrict__ bp, const int2 *__restrict__ map,
                                                   int role_x, int role_b, int role_r, int use_skip) {
    extern __shared__ unsigned char smem_raw[];
    const int2 m = map[blockIdx.x];
    const BatchProb &q = bp[m.x];
    using TS = TileShape<2, P>;
    int bx, by;
    xcd_relabel(m.y, q.res_ntx, q.res_ntx * q.res_nty, bx, by);
    constexpr int pr = prec_slot<T>();
    residual_body<2, P, T, NORM>(static_cast<const T *>(q.val[pr]), q.npad, q.pitch1, 0, q.n1, TS::TX, TS::TY, 1,
                                 static_cast<const T *>(q.vec[role_x]), static_cast<const T *>(q.vec[role_b]),
                                 static_cast<T *>(q.vec[role_r]), NORM ? q.partial + m.y : nullptr,
                                 static_cast<const T *>(q.cs[pr]), q.ulo, q.uhi, use_skip ? q.flags : nullptr, bx,
                                 by, 0, reinterpret_cast<T *>(smem_raw), static_cast<const T *>(q.fac[pr]));
}

__global__ void __launch_bounds__(256) kb_norm_finalize(const BatchProb *__restrict__ bp, int scale_fp32, int book) {
    const BatchProb &q = bp[blockIdx.x];
    finalize_body(q.partial, q.res_ntx * q.res_nty, q.scal, scale_fp32, book ? q.flags : nullptr, q.hist, q.hist_cap);
}

__global__ void kb_solve_init(const BatchProb *__restrict__ bp, int nprob, double tol, int max_cycles) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nprob) init_body(bp[i].scal, bp[i].flags, tol, max_cycles);
}

// colour (cx, cy) of period S; the tile grid of every problem covers the
// grids of all colours, so tiles past the end of a colour's grid do nothing
template <int P, int B, class T>
__global__ void __launch_bounds__(kColourThreads) kb_colour(const BatchProb *__restrict__ bp, const int2 *__restrict__ map,
                                                  int nbx, int nby, int cx, int cy, int S, int role_src, int role_dst,
                                                  int role_rhs, int x_zero, int fuse, int use_skip) {
    extern __shared__ unsigned char smem_raw[];
    const int2 m = map[blockIdx.x];
    const BatchProb &q = bp[m.x];
    constexpr int HB = (B - 1) / 2;
    int ox = cx - HB, oy = cy - HB;
    if (ox > 0) ox -= S;
    if (oy > 0) oy -= S;
    const int bx = m.y % q.col_ntx, by = m.y / q.col_ntx;
    if (ox + bx * nbx * S >= q.n1 || oy + by * nby * S >= q.n1) return;
    constexpr int pr = prec_slot<T>();
    colour_body<2, P, B, T, false>(static_cast<const T *>(q.val[pr]), q.npad, q.pitch1, 0, q.n1,
                            static_cast<const T *>(q.inv[pr]), q.clsL, q.ncls1, static_cast<const T *>(q.vec[role_src]),
                            static_cast<T *>(q.vec[role_dst]), static_cast<const T *>(q.vec[role_rhs]), x_zero, ox, oy,
                            0, S, nbx, nby, 1, static_cast<const T *>(q.cs[pr]), q.ulo, q.uhi,
                            use_skip ? q.flags : nullptr,
                            fuse ? static_cast<const double *>(q.vec[kVecR64]) : nullptr, q.scal,
                            fuse ? static_cast<T *>(q.vec[kVecRhsW]) : nullptr, bx, by, 0, smem_raw,
                            static_cast<const T *>(q.fac[pr]));
}

}  // namespace

// ------------------------------------------------------------ launchers --
void launch_residual64(const Problem &Pb, const double *u, const double *b, double *r, bool with_norm,
                       bool scale_fp32, bool book, hipStream_t s) {
    if (Pb.dim == 2) {
        IGA2L_DISPATCH_P2(res64_dp, Pb, u, b, r, with_norm, scale_fp32, book, s);
    } else {
        IGA2L_DISPATCH_P3(res64_dp, Pb, u, b, r, with_norm, scale_fp32, book, s);
    }
}

template <class T>
void launch_defect(const Problem &Pb, const T *e, const T *rhs, T *d, hipStream_t s) {
    if (Pb.dim == 2) {
        IGA2L_DISPATCH_P2(defect_dp, Pb, e, rhs, d, s);
    } else {
        IGA2L_DISPATCH_P3(defect_dp, Pb, e, rhs, d, s);
    }
}
template void launch_defect<double>(const Problem &, const double *, const double *, double *, hipStream_t);
template void launch_defect<float>(const Problem &, const float *, const float *, float *, hipStream_t);

// number of workgroups of the FP64 residual launch (one partial sum each)
int64_t residual_workgroups(const Problem &Pb) {
    if (residual3d_sf_ok(Pb)) return residual3d_sf_workgroups(Pb);
    if (Pb.dim == 2 && Pb.fine.n >= (int64_t(1) << 20)) return residual2d_workgroups(Pb);
    const int64_t n1 = Pb.fine.n1;
    if (Pb.dim == 2) return ((n1 + TileShape<2, 1>::TX - 1) / TileShape<2, 1>::TX) * ((n1 + TileShape<2, 1>::TY - 1) / TileShape<2, 1>::TY);
    return ((n1 + TileShape<3, 1>::TX - 1) / TileShape<3, 1>::TX) * ((n1 + TileShape<3, 1>::TY - 1) / TileShape<3, 1>::TY) *
           ((n1 + TileShape<3, 1>::TZ - 1) / TileShape<3, 1>::TZ);
}

void launch_solve_init(const Problem &Pb, double tol, int max_cycles, hipStream_t s) {
    hipLaunchKernelGGL(k_solve_init, dim3(1), dim3(64), 0, s, Pb.scal.as<double>(), dev_flags(Pb), tol, max_cycles);
}


template <class T>
void launch_colour_step(const Problem &Pb, int cx, int cy, int cz, int S, const T *x_src, T *x_dst, const T *rhs,
                        bool x_zero, hipStream_t s, const double *r64, T *rhs_out) {
    IGA2L_REQUIRE(!r64 || (x_zero && rhs_out), IGA2L_EINVAL, "fused cast needs a zero iterate and an output");
    if (Pb.dim == 2) {
        IGA2L_DISPATCH_P2(colour_dp, Pb, cx, cy, cz, S, x_src, x_dst, rhs, x_zero, r64, rhs_out, s);
    } else {
        IGA2L_DISPATCH_P3(colour_dp, Pb, cx, cy, cz, S, x_src, x_dst, rhs, x_zero, r64, rhs_out, s);
    }
}
template void launch_colour_step<double>(const Problem &, int, int, int, int, const double *, double *,
                                         const double *, bool, hipStream_t, const double *, double *);
template void launch_colour_step<float>(const Problem &, int, int, int, int, const float *, float *, const float *,
                                        bool, hipStream_t, const double *, float *);

bool lex_sweep_fits(const Problem &Pb) {
    const int64_t bd = (Pb.dim == 3) ? int64_t(Pb.bw) * Pb.bw * Pb.bw : int64_t(Pb.bw) * Pb.bw;
    return !Pb.lex_off.empty() && int64_t(Pb.lex_maxcnt) * bd <= kLexThreads && lex_sweep_lds(Pb) <= 64 * 1024;
}

void launch_lex_sweep(const Problem &Pb, double *u, const double *b, hipStream_t s) {
    IGA2L_REQUIRE(lex_sweep_fits(Pb), IGA2L_EUNSUPPORTED, "grid too large for the one-workgroup sweep");
    if (Pb.dim == 2) {
        IGA2L_DISPATCH_P2(lex_sweep_dp, Pb, u, b, s);
    } else {
        IGA2L_DISPATCH_P3(lex_sweep_dp, Pb, u, b, s);
    }
}

void launch_lex_step(const Problem &Pb, int step, double *u, const double *b, hipStream_t s) {
    if (Pb.dim == 2) {
        IGA2L_DISPATCH_P2(lex_dp, Pb, step, u, b, s);
    } else {
        IGA2L_DISPATCH_P3(lex_dp, Pb, step, u, b, s);
    }
}

template <class T>
void launch_cast_scale(const Problem &Pb, const double *r64, T *rhs, hipStream_t s) {
    const int64_t n = Pb.fine.n;
    hipLaunchKernelGGL((k_cast_scale<T>), dim3((n + 255) / 256), dim3(256), 0, s, r64, rhs, Pb.scal.as<double>(), n,
                       Pb.skip);
}
template void launch_cast_scale<float>(const Problem &, const double *, float *, hipStream_t);
template void launch_cast_scale<double>(const Problem &, const double *, double *, hipStream_t);

void launch_block_inverse(Problem &Pb, const std::vector<int64_t> &reps, hipStream_t s) {
    DevBuf reps_d;
    reps_d.alloc(reps.size() * sizeof(int64_t));
    IGA2L_HIP(hipMemcpyAsync(reps_d.ptr, reps.data(), reps.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    DevBuf err;
    err.alloc(sizeof(int));
    IGA2L_HIP(hipMemsetAsync(err.ptr, 0, sizeof(int), s));
    const unsigned nblk = unsigned(reps.size());
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(nblk), dim3(kWave), 0, s, Pb.A.v64.as<double>(), Pb.A.npad, Pb.A.pitch[1],
                           Pb.A.pitch[2], Pb.fine.n1, Pb.p, reps_d.as<int64_t>(), Pb.Inv64.as<double>(), err.as<int>());
    };
    if (Pb.dim == 2) {
        switch (Pb.bw) {
            case 1: go(k_block_inverse<2, 1>); break;
            case 3: go(k_block_inverse<2, 3>); break;
            case 5: go(k_block_inverse<2, 5>); break;
            case 7: go(k_block_inverse<2, 7>); break;
            default: throw Error{IGA2L_EUNSUPPORTED, "block width must be 1, 3, 5 or 7"};
        }
    } else {
        switch (Pb.bw) {
            case 1: go(k_block_inverse<3, 1>); break;
            case 3: go(k_block_inverse<3, 3>); break;
            default: throw Error{IGA2L_EUNSUPPORTED, "3-D block width must be 1 or 3"};
        }
    }
    IGA2L_HIP(hipGetLastError());
    int herr = 0;
    IGA2L_HIP(hipMemcpyAsync(&herr, err.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    IGA2L_HIP(hipStreamSynchronize(s));
    IGA2L_REQUIRE(herr == 0, IGA2L_ENUMERIC, "a Schwarz block matrix is not positive definite");
}

// ------------------------------------------------------- batched launchers --
void colour_tile_clamp(int S, int &nbx, int &nby) {
    while (nbx * S * nby * S > kColourThreads) {
        if (nby > 1) --nby;
        else if (nbx > 1) --nbx;
        else break;
    }
}

size_t colour_lds(int p, int S, int nbx, int nby, size_t elem, bool factor_rows) {
    const size_t TX = size_t(nbx) * S, TY = size_t(nby) * S, W = size_t(2 * p + 1) * (2 * p + 1);
    const size_t sf2 = factor_rows ? 2 * (TY + 2 * p) * TX : 0;
    return ((TX + 2 * p) * (TY + 2 * p) + TX * TY + W + sf2) * elem;
}

const void *colour_factor_rows(const Problem &P, bool fp64) {
    if (P.dim != 2) return nullptr;
    if (P.geometry == kGeomAnnulus) return fp64 ? P.fac2d64.ptr : P.fac2d32.ptr;
    // kappa = 1 square: measured faster than the stencil and stored diagonals
    // on the latency-bound grids (the wavefronts next to the boundary no
    // longer read (2p+1)^2 diagonals); the large tiled instance keeps them
    if (P.fine.n >= kColourPreMaxN) return nullptr;
    return fp64 ? P.fac64.ptr : P.fac32.ptr;
}

template <int P, class T, bool NORM>
void launch_residual_batch(const BatchProb *bp, const int2 *map, int nwg, int role_x, int role_b, int role_r,
                           bool use_skip, hipStream_t s) {
    using TS = TileShape<2, P>;
    const size_t shm = (size_t(TS::TX + 2 * P) * (TS::TY + 2 * P) + size_t(2 * P + 1) * (2 * P + 1)) * sizeof(T);
    hipLaunchKernelGGL((kb_residual<P, T, NORM>), dim3(nwg), dim3(TS::TX * TS::TY), shm, s, bp, map, role_x, role_b,
                       role_r, use_skip ? 1 : 0);
}

template <class T>
void launch_residual_batch_dispatch(int p, const BatchProb *bp, const int2 *map, int nwg, int role_x, int role_b,
                                    int role_r, bool norm, bool use_skip, hipStream_t s) {
#define IGA2L_RB_CASE(PP)                                                                                 \
    case PP:                                                                                              \
        if (norm) launch_residual_batch<PP, T, true>(bp, map, nwg, role_x, role_b, role_r, use_skip, s);  \
        else launch_residual_batch<PP, T, false>(bp, map, nwg, role_x, role_b, role_r, use_skip, s);      \
        break;
    switch (p) {
        IGA2L_RB_CASE(1)
        IGA2L_RB_CASE(2)
        IGA2L_RB_CASE(3)
        IGA2L_RB_CASE(4)
        IGA2L_RB_CASE(5)
        IGA2L_RB_CASE(6)
        IGA2L_RB_CASE(7)
        IGA2L_RB_CASE(8)
        default: throw Error{IGA2L_EUNSUPPORTED, "degree out of range"};
    }
#undef IGA2L_RB_CASE
}
template void launch_residual_batch_dispatch<double>(int, const BatchProb *, const int2 *, int, int, int, int, bool,
                                                     bool, hipStream_t);
template void launch_residual_batch_dispatch<float>(int, const BatchProb *, const int2 *, int, int, int, int, bool,
                                                    bool, hipStream_t);

void launch_norm_finalize_batch(const BatchProb *bp, int nprob, bool scale_fp32, bool book, hipStream_t s) {
    hipLaunchKernelGGL(kb_norm_finalize, dim3(nprob), dim3(256), 0, s, bp, scale_fp32 ? 1 : 0, book ? 1 : 0);
}

void launch_solve_init_batch(const BatchProb *bp, int nprob, double tol, int max_cycles, hipStream_t s) {
    hipLaunchKernelGGL(kb_solve_init, dim3((nprob + 63) / 64), dim3(64), 0, s, bp, nprob, tol, max_cycles);
}

template <class T>
void launch_colour_batch(const BatchProb *bp, const int2 *map, int nwg, int p, int bw, int nbx, int nby, int cx,
                         int cy, int S, int role_src, int role_dst, int role_rhs, bool x_zero, bool fuse,
                         hipStream_t s, bool use_skip) {
    const int threads = ((nbx * S * nby * S + kWave - 1) / kWave) * kWave;
    // (room for the factor rows' x sums: some problems of the table may use them)
    const size_t shm = colour_lds(p, S, nbx, nby, sizeof(T), true);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(nwg), dim3(threads), shm, s, bp, map, nbx, nby, cx, cy, S, role_src, role_dst,
                           role_rhs, x_zero ? 1 : 0, fuse ? 1 : 0, use_skip ? 1 : 0);
    };
#define IGA2L_CB_P(PP)                                                           \
    case PP:                                                                     \
        switch (bw) {                                                            \
            case 1: go(kb_colour<PP, 1, T>); break;                              \
            case 3: go(kb_colour<PP, 3, T>); break;                              \
            case 5: go(kb_colour<PP, 5, T>); break;                              \
            case 7: go(kb_colour<PP, 7, T>); break;                              \
            default: throw Error{IGA2L_EUNSUPPORTED, "block width must be 1, 3, 5 or 7"}; \
        }                                                                        \
        break;
    switch (p) {
        IGA2L_CB_P(1)
        IGA2L_CB_P(2)
        IGA2L_CB_P(3)
        IGA2L_CB_P(4)
        IGA2L_CB_P(5)
        IGA2L_CB_P(6)
        IGA2L_CB_P(7)
        IGA2L_CB_P(8)
        default: throw Error{IGA2L_EUNSUPPORTED, "degree out of range"};
    }
#undef IGA2L_CB_P
}
template void launch_colour_batch<double>(const BatchProb *, const int2 *, int, int, int, int, int, int, int, int,
                                          int, int, int, bool, bool, hipStream_t, bool);
template void launch_colour_batch<float>(const BatchProb *, const int2 *, int, int, int, int, int, int, int, int, int,
                                         int, int, bool, bool, hipStream_t, bool);

// -------------------------------------------------------------- autotuner --
bool tune_log() {
    static const bool on = [] {
        const char *v = std::getenv("IGA2L_TUNE_LOG");
        return v && *v && *v != '0';
    }();
    return on;
}

std::vector<std::pair<int, int>> colour_tile_candidates(int S, int n1) {
    // the last rows serve long colour periods (s = b + p up to 15: a cell of s x s points)
    static const int shapes[][2] = {{4, 4}, {8, 2}, {8, 4},  {16, 1}, {16, 2}, {16, 4}, {32, 1}, {32, 2},
                                    {4, 8}, {11, 3}, {22, 2}, {28, 2}, {43, 1}, {12, 4}, {64, 1},
                                    {1, 1}, {2, 1}, {1, 2}, {2, 2}, {3, 1}, {4, 1}, {3, 2}, {4, 2}};
    std::vector<std::pair<int, int>> out;
    const int cells = (n1 + 2 * S - 1) / S;   // cells a colour's grid spans per direction
    for (auto &sh : shapes) {
        const int bx = sh[0], by = sh[1];
        if (bx * S * by * S > kColourThreads || bx * S * by * S < 64) continue;
        if (bx > cells + 1 && !(bx == 4 && by == 4)) continue;   // wider than the grid
        out.emplace_back(bx, by);
    }
    return out;
}

template <class T>
void autotune_colour_tile(Problem &Pb, int S, hipStream_t s) {
    if (Pb.dim != 2) return;
    constexpr int pr = std::is_same<T, double>::value ? 0 : 1;
    const T *rhs = std::is_same<T, double>::value ? reinterpret_cast<const T *>(Pb.r64.ptr)
                                                  : reinterpret_cast<const T *>(Pb.rhs_w.ptr);
    const T *src = Pb.ework[0].as<T>();
    T *dst = Pb.ework[1].as<T>();
    const int *saved = Pb.skip;
    Pb.skip = nullptr;
    hipEvent_t e0, e1;
    IGA2L_HIP(hipEventCreate(&e0));
    IGA2L_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int bbx = Pb.tile_bx[pr], bby = Pb.tile_by[pr];
    const int reps = 3;
    try {
        for (auto [cbx, cby] : colour_tile_candidates(S, Pb.fine.n1)) {
            // the middle colour; warm-up launch, then timed launches
            IGA2L_DISPATCH_P2(colour_dp, Pb, 1, 1, 0, S, src, dst, rhs, false, nullptr, static_cast<T *>(nullptr), s,
                              cbx, cby);
            IGA2L_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r)
                IGA2L_DISPATCH_P2(colour_dp, Pb, 1, 1, 0, S, src, dst, rhs, false, nullptr,
                                  static_cast<T *>(nullptr), s, cbx, cby);
            IGA2L_HIP(hipEventRecord(e1, s));
            IGA2L_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            IGA2L_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (tune_log())
                std::fprintf(stderr, "[iga2l tune] p=%d n1=%d s=%d %s: tile %dx%d blocks %.2f us\n", Pb.p, Pb.fine.n1,
                             S, pr ? "fp32" : "fp64", cbx, cby, 1e3f * ms / reps);
            if (ms < best) {
                best = ms;
                bbx = cbx;
                bby = cby;
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        Pb.skip = saved;
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    Pb.skip = saved;
    Pb.tile_bx[pr] = bbx;
    Pb.tile_by[pr] = bby;
}
template void autotune_colour_tile<double>(Problem &, int, hipStream_t);
template void autotune_colour_tile<float>(Problem &, int, hipStream_t);

}  // namespace iga2l
