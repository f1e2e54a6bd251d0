// kernels_2d.hip -- bandwidth-oriented 2-D kernels of the two-level cycle:
// the wide-band residual with register blocking along y, and the restriction
// and prolongation as two 1-D passes (the transfer is R1 (x) R1, so a coarse
// value needs p+2 taps per direction instead of (p+2)^2 gathers).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "internal.h"

namespace iga2l {

// transfer tiles: 64 x 16 points on large grids, 32 x 8 otherwise
void transfer_tile_2d(int64_t n1, int &tx, int &ty) {
    if (n1 >= 1024) { tx = 64; ty = 16; }
    else { tx = 32; ty = 8; }
}

namespace {

inline unsigned nblk(int64_t n, int t) { return unsigned((n + t - 1) / t); }


// ------------------------------------------------------------------------
// shared pieces of the 2-D residual kernels
constexpr int kResTX = 64, kResTYT = 4, kResRY = 4, kResCH = kResTYT * kResRY, kResRing = 32;
constexpr int kResTargetGroups = 8192;  // about four rounds of the resident workgroups

// the workgroup's sum of rr (a fixed order: wavefront reductions, then the
// wavefronts in turn), written by thread 0
template <int NT>
__device__ __forceinline__ void block_partial(double rr, double *out) {
    __shared__ double red[NT / 64];
    for (int off = 32; off > 0; off >>= 1) rr += __shfl_down(rr, off, 64);
    if ((threadIdx.x % 64) == 0) red[threadIdx.x / 64] = rr;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < NT / 64; ++k) s += red[k];
        *out = s;
    }
}

// r = b - A x at frame point f (kappa = 1): the points with a coordinate
// outside [ulo, uhi], numbered by the bands above and below the interior rows
// (whole grid rows), then by the rows in between (their ulo + (n1-1-uhi)
// outer columns).  The row of A is K1 (x) M1 + M1 (x) K1 of the point's own
// 1-D rows (fac: K1 then M1, [n1][2P+1] each), applied by sum factorisation
// like the interior stencil; entries that would leave the grid are zero in
// the 1-D rows.
template <int P, class T>
__device__ __forceinline__ void residual_frame_point(const T *__restrict__ fac, int n1, int ulo, int uhi, int64_t f,
                                                     const T *__restrict__ x, const T *__restrict__ b,
                                                     T *__restrict__ r, double &rr) {
    constexpr int W1 = 2 * P + 1;
    const int L = ulo, R = n1 - 1 - uhi, LR = L + R;
    const int64_t nband = int64_t(LR) * n1, nf = nband + int64_t(uhi - ulo + 1) * LR;
    if (f >= nf) return;
    int gx, gy;
    if (f < nband) {
        const int row = int(f / n1);
        gx = int(f % n1);
        gy = row < L ? row : uhi + 1 + (row - L);
    } else {
        const int64_t g = f - nband;
        const int c = int(g % LR);
        gy = ulo + int(g / LR);
        gx = c < L ? c : uhi + 1 + (c - L);
    }
    const T *K = fac, *M = fac + int64_t(n1) * W1;
    const T *Kx = K + int64_t(gx) * W1, *Mx = M + int64_t(gx) * W1;
    const T *Ky = K + int64_t(gy) * W1, *My = M + int64_t(gy) * W1;
    T acc = T(0);
    // every load in flight at once for P <= 3; a run-time loop over the
    // stencil rows above, where the unrolled loads would set the register
    // count of the whole kernel
#pragma unroll(P <= 3 ? W1 : 1)
    for (int oy = 0; oy < W1; ++oy) {
        const int jy = min(max(gy + oy - P, 0), n1 - 1);
        T mx = T(0), kx = T(0);
#pragma unroll
        for (int ox = 0; ox < W1; ++ox) {
            const int jx = min(max(gx + ox - P, 0), n1 - 1);
            // clamped reads: the factor entry of a neighbour outside the grid is zero
            const T v = x[int64_t(jy) * n1 + jx];
            kx += Kx[ox] * v;
            mx += Mx[ox] * v;
        }
        acc += Ky[oy] * mx + My[oy] * kx;
    }
    const int64_t gi = int64_t(gy) * n1 + gx;
    const T res = b[gi] - acc;
    r[gi] = res;
    rr = double(res) * double(res);
}

// ------------------------------------------------------------------------
// r = b - A x for a variable coefficient, on tiles of 64 x (4*RY) points.
// Each thread owns a column of RY consecutive points (x fixed); the LDS rows
// it needs are read once into registers and reused by every output of the
// column they touch, and the (2P+1)^2 diagonals of each output are read with
// all their loads in flight together.

template <int P, class T, bool NORM>
__global__ void __launch_bounds__(kResTX *kResTYT) k_residual2d_tiled(const T *__restrict__ val, int64_t npad, int pitch1,
                                                                int n1, const T *__restrict__ x,
                                                                const T *__restrict__ b, T *__restrict__ r,
                                                                double *__restrict__ partial,
                                                                const int *__restrict__ skip) {
    constexpr int TX = kResTX, TY = kResTYT * kResRY, RY = kResRY;
    constexpr int HX = TX + 2 * P, HY = TY + 2 * P;
    constexpr int W1 = 2 * P + 1, W = W1 * W1, C0 = (W - 1) / 2;
    constexpr int NT = kResTX * kResTYT;
    __shared__ T xs[HX * HY];
    if (skip && *skip) return;
    int bx, by;
    xcd_tile_2d(bx, by);
    const int gx0 = bx * TX, gy0 = by * TY;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int gx = gx0 + tx, gyb = gy0 + ty * RY;
    // the whole halo in one round trip
    stage_lds<(HX * HY + NT - 1) / NT>(xs, HX * HY, [&](int h) {
        const int hx = h % HX, hy = h / HX;
        const int hgx = gx0 + hx - P, hgy = gy0 + hy - P;
        return (hgx >= 0 && hgx < n1 && hgy >= 0 && hgy < n1) ? x[int64_t(hgy) * n1 + hgx] : T(0);
    });
    __syncthreads();
    T acc[RY];
#pragma unroll
    for (int k = 0; k < RY; ++k) acc[k] = T(0);
    if (gx < n1) {
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int gy = gyb + k;
            if (gy >= n1) continue;
            const int64_t padi = int64_t(gx + P) + int64_t(gy + P) * pitch1;
#pragma unroll
            for (int oy = 0; oy < W1; ++oy)
#pragma unroll
                for (int ox = 0; ox < W1; ++ox) {
                    const int w = oy * W1 + ox;
                    const T a = (w >= C0) ? val[int64_t(w - C0) * npad + padi]
                                          : val[int64_t(C0 - w) * npad + padi + (ox - P) + int64_t(oy - P) * pitch1];
                    acc[k] += a * xs[(ty * RY + k + oy) * HX + tx + ox];
                }
        }
    }
    double rr = 0.0;
    if (gx < n1) {
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int gy = gyb + k;
            if (gy < n1) {
                const int64_t gi = int64_t(gy) * n1 + gx;
                const T res = b[gi] - acc[k];
                r[gi] = res;
                rr += double(res) * double(res);
            }
        }
    }
    if constexpr (NORM) {
        __shared__ double red[kResTX * kResTYT / 64];
        for (int off = 32; off > 0; off >>= 1) rr += __shfl_down(rr, off, 64);
        if ((threadIdx.x % 64) == 0) red[threadIdx.x / 64] = rr;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int k = 0; k < int(blockDim.x / 64); ++k) s += red[k];
            partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
        }
    }
}


// ------------------------------------------------------------------------
// r = b - A x for kappa = 1, streamed.  Points whose coordinates all lie in
// [ulo, uhi] carry the interior stencil, K1 (x) M1 + M1 (x) K1 of the interior
// 1-D rows cf (K1 then M1), applied by sum factorisation (per window row the x
// sums of both factors, then the y taps).  A workgroup owns a strip of 64
// columns over a segment of rows and walks down it in chunks of 16 rows; a
// thread owns a column of RY consecutive points of the chunk.  The x window
// lives in an LDS ring of 32 rows, so the 2P halo rows shared by consecutive
// chunks are read from memory once, and the rows of the next chunk (and its
// right-hand side) are loaded into registers while the current chunk
// computes, which keeps memory requests in flight through the arithmetic.
// The first workgroups of the grid instead take the frame of points within
// ulo of the boundary, one point per thread, from the 1-D rows of the factors.

template <int P, class T, bool NORM>
__global__ void __launch_bounds__(kResTX *kResTYT, (sizeof(T) == 8 && P == 8) ? 3 : 4)
    k_residual2d(const T *__restrict__ fac, int n1, int nframe_groups, int nsx, int nseg, int seg_rows,
                 const T *__restrict__ x, const T *__restrict__ b, T *__restrict__ r, double *__restrict__ partial,
                 const T *__restrict__ cf, int ulo, int uhi, const int *__restrict__ skip) {
    constexpr int TX = kResTX, CH = kResCH, RY = kResRY, RING = kResRing;
    constexpr int HX = TX + 2 * P;
    constexpr int W1 = 2 * P + 1, NT = kResTX * kResTYT;
    static_assert(CH + 2 * P <= RING && (RING & (RING - 1)) == 0, "ring: a power of two holding the window");
    __shared__ T ring[RING * HX];
    if (skip && *skip) return;
    const int id = int(blockIdx.x);
    const int tid = int(threadIdx.x);
    double rr = 0.0;
    if (id < nframe_groups) {
        residual_frame_point<P, T>(fac, n1, ulo, uhi, int64_t(id) * NT + tid, x, b, r, rr);
        if constexpr (NORM) block_partial<NT>(rr, partial + id);
        return;
    }
    // nframe_groups is a multiple of the XCD count: strip workgroups keep the
    // XCD-banded tile order of a grid of their own
    int bx, bs;
    xcd_relabel(id - nframe_groups, nsx, nsx * nseg, bx, bs);
    const int gx0 = bx * TX, y0 = bs * seg_rows;
    const int y1 = min(y0 + seg_rows, n1);
    const int nch = (y1 - y0 + CH - 1) / CH;
    const int tx = tid % TX, ty = tid / TX;
    const int gx = gx0 + tx;
    // window row q (0-based from global row y0 - P) sits in ring slot q % RING,
    // window column hx at global column gx0 - P + hx
    // the 2P rows above the first chunk
    stage_lds<(2 * P * HX + NT - 1) / NT>(ring, 2 * P * HX, [&](int h) {
        const int hgx = gx0 + h % HX - P, hgy = y0 - P + h / HX;
        return (hgx >= 0 && hgx < n1 && hgy >= 0 && hgy < n1) ? x[int64_t(hgy) * n1 + hgx] : T(0);
    });
    // rows 2P .. CH+2P-1 of chunk c's window are new (global rows y0 + c CH + P + j):
    // the 64 columns of the strip, row ty + 4u for thread (tx, ty), and the 2P
    // halo columns, thread t taking row t % CH of halo column t / CH.  Loads
    // read clamped addresses, unpredicated; positions outside the grid are
    // zeroed where the values enter the ring, so no instruction consumes a
    // loaded value before the chunk's arithmetic is done.
    constexpr int NI = CH / kResTYT, NH = (2 * P * CH + NT - 1) / NT;
    const int gxc = min(gx, n1 - 1);
    T xi[NI], xh[NH];
    auto halo_col = [&](int hc) { return hc < P ? gx0 - P + hc : gx0 + TX - P + hc; };
    auto prefetch = [&](int c) {
        const int ybase = y0 + c * CH + P;
#pragma unroll
        for (int u = 0; u < NI; ++u) xi[u] = x[int64_t(min(ybase + ty + kResTYT * u, n1 - 1)) * n1 + gxc];
#pragma unroll
        for (int u = 0; u < NH; ++u) {
            const int t = tid + u * NT;
            const int gxh = halo_col(t / CH);
            xh[u] = x[int64_t(min(ybase + t % CH, n1 - 1)) * n1 + min(max(gxh, 0), n1 - 1)];
        }
    };
    auto store_ring = [&](int c) {
        const int q = c * CH + 2 * P, ybase = y0 + c * CH + P;
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            const int j = ty + kResTYT * u;
            ring[((q + j) & (RING - 1)) * HX + P + tx] = (gx < n1 && ybase + j < n1) ? xi[u] : T(0);
        }
#pragma unroll
        for (int u = 0; u < NH; ++u) {
            const int t = tid + u * NT, j = t % CH, hc = t / CH;
            const int gxh = halo_col(hc);
            if (t < 2 * P * CH)
                ring[((q + j) & (RING - 1)) * HX + (hc < P ? hc : TX + hc)] =
                    (gxh >= 0 && gxh < n1 && ybase + j < n1) ? xh[u] : T(0);
        }
    };
    // the right-hand side of the column (read where the output exists only)
    T bv[RY], bn[RY];
    auto prefetch_b = [&](int c, T *dst) {
#pragma unroll
        for (int k = 0; k < RY; ++k) dst[k] = b[int64_t(min(y0 + c * CH + ty * RY + k, n1 - 1)) * n1 + gxc];
    };
    prefetch_b(0, bv);
    prefetch(0);
    store_ring(0);
    __syncthreads();
    const bool col_in = gx >= ulo && gx <= uhi;
    // per chunk: issue the next chunk's loads (right-hand side first), compute
    // from the ring, move the loaded rows in once every wavefront is done with
    // the ring, and only then store the results.  Each wait is on loads issued
    // before the arithmetic, and every store is older than the loads waited
    // on next, so neither the stores nor the next loads stall a chunk.
    for (int c = 0; c < nch; ++c) {
        const bool more = c + 1 < nch;
        if (more) {
            prefetch_b(c + 1, bn);
            prefetch(c + 1);
        }
        const int gyb = y0 + c * CH + ty * RY;
        const int q0 = c * CH + ty * RY;  // window row of the column's first point, minus P
        T acc[RY];
#pragma unroll
        for (int k = 0; k < RY; ++k) acc[k] = T(0);
        // (threads whose rows all lie past the segment have nothing to compute;
        // keeping the arithmetic under this chunk-dependent test also keeps
        // the compiler from holding the whole unrolled window in registers)
        if (gyb < y1) {
            // row yy of the column window (0 .. RY+2P-1) feeds output k with oy = yy - k
#pragma unroll
            for (int yy = 0; yy < RY + 2 * P; ++yy) {
                const T *row = ring + ((q0 + yy) & (RING - 1)) * HX + tx;
                T mx = T(0), kx = T(0);
#pragma unroll
                for (int ox = 0; ox < W1; ++ox) {
                    const T v = row[ox];
                    kx += cf[ox] * v;
                    mx += cf[W1 + ox] * v;
                }
#pragma unroll
                for (int k = 0; k < RY; ++k) {
                    const int oy = yy - k;
                    if (oy >= 0 && oy < W1) acc[k] += cf[oy] * mx + cf[W1 + oy] * kx;
                }
            }
        }
        if (more) {
            __syncthreads();  // the next chunk's rows overwrite slots this one read
            store_ring(c + 1);
            __syncthreads();
        }
        if (col_in) {
#pragma unroll
            for (int k = 0; k < RY; ++k) {
                const int gy = gyb + k;
                if (gy < y1 && gy >= ulo && gy <= uhi) {
                    const T res = bv[k] - acc[k];
                    r[int64_t(gy) * n1 + gx] = res;
                    rr += double(res) * double(res);
                }
            }
        }
        if (more) {
#pragma unroll
            for (int k = 0; k < RY; ++k) bv[k] = bn[k];
        }
    }
    if constexpr (NORM) block_partial<NT>(rr, partial + id);
}

int stream_segment_rows(int64_t n1, int tx, int ch, int64_t target, const char *env);

// rows per segment of the streamed residual (the environment variable
// IGA2L_RESIDUAL_GROUPS sets another workgroup target: tests use a small one
// to send many chunks through each ring)
int residual2d_segment_rows(int64_t n1) {
    return stream_segment_rows(n1, kResTX, kResCH, kResTargetGroups, "IGA2L_RESIDUAL_GROUPS");
}

// ------------------------------------------------------------------------
// d_c = (R1 (x) R1) d on tiles of CX x CY coarse points.  Coarse I uses fine
// I-1 .. I+p per direction.  Pass 1 (x): t[row][I] for every fine row of the
// window; pass 2 (y): d_c[J][I].  The 1-D factor rows of the tile are staged.
// transfer tiles: 64 x 16 on large grids, 32 x 8 where that would leave the
// device under-occupied

template <class T>
__device__ __forceinline__ void restrict2d_body(const T *__restrict__ R1, int p, int n1f, int n1c,
                                                const T *__restrict__ df, T *__restrict__ dc,
                                                const int *__restrict__ skip, int CX, int CY, int bx, int by,
                                                T *sm) {
    const int w = p + 2;
    const int FX = CX + p + 1, FY = CY + p + 1;        // fine window (I0-1 .. I0+CX-1+p)
    T *ds = sm;                                          // [FY][FX]
    T *ts = ds + FX * FY;                                // [FY][CX]
    T *rx = ts + FY * CX;                                // [CX][w]
    T *ry = rx + CX * w;                                 // [CY][w]
    const int stop = skip ? *skip : 0;
    const int I0 = bx * CX, J0 = by * CY;
    // the fine window in one memory round trip (at most 8 loads per thread:
    // 64 x 16 coarse tiles of p <= 8 with 256 threads)
    stage_lds<8>(ds, FX * FY, [&](int h) {
        const int hx = h % FX, hy = h / FX;
        const int jx = I0 - 1 + hx, jy = J0 - 1 + hy;
        return (jx >= 0 && jx < n1f && jy >= 0 && jy < n1f) ? df[int64_t(jy) * n1f + jx] : T(0);
    });
    for (int h = threadIdx.x; h < CX * w; h += blockDim.x) {
        const int I = I0 + h / w;
        rx[h] = (I < n1c) ? R1[int64_t(I) * w + h % w] : T(0);
    }
    for (int h = threadIdx.x; h < CY * w; h += blockDim.x) {
        const int J = J0 + h / w;
        ry[h] = (J < n1c) ? R1[int64_t(J) * w + h % w] : T(0);
    }
    __syncthreads();
    for (int h = threadIdx.x; h < FY * CX; h += blockDim.x) {
        const int cx = h % CX, fy = h / CX;
        T acc = T(0);
        for (int a = 0; a < w; ++a) acc += rx[cx * w + a] * ds[fy * FX + cx + a];
        ts[fy * CX + cx] = acc;
    }
    __syncthreads();
    if (stop) return;
    for (int h = threadIdx.x; h < CX * CY; h += blockDim.x) {
        const int cx = h % CX, cy = h / CX;
        const int I = I0 + cx, J = J0 + cy;
        if (I >= n1c || J >= n1c) continue;
        T acc = T(0);
        for (int bb = 0; bb < w; ++bb) acc += ry[cy * w + bb] * ts[(cy + bb) * CX + cx];
        dc[int64_t(J) * n1c + I] = acc;
    }
}

template <class T>
__global__ void __launch_bounds__(256) k_restrict2d(const T *__restrict__ R1, int p, int n1f, int n1c,
                                                    const T *__restrict__ df, T *__restrict__ dc,
                                                    const int *__restrict__ skip, int CX, int CY) {
    extern __shared__ unsigned char smem_raw[];
    int bx, by;
    xcd_tile_2d(bx, by);
    restrict2d_body<T>(R1, p, n1f, n1c, df, dc, skip, CX, CY, bx, by, reinterpret_cast<T *>(smem_raw));
}

// ------------------------------------------------------------------------
// (R1 (x) R1)^T e_c on tiles of TX x TY fine points; fine i takes coarse
// I = i-p .. i+1 with weight R1[I][i-I+1].  mode 0: uf += P e_c;  mode 1:
// u64 += sigma (e + P e_c) (end of a correction cycle; sigma from scal when
// scaled).
template <class T>
__device__ __forceinline__ void prolong2d_body(const T *__restrict__ R1, int p, int n1f, int n1c,
                                               const T *__restrict__ ec, T *__restrict__ uf, int mode,
                                               const T *__restrict__ e, double *__restrict__ u64,
                                               const double *__restrict__ scal, int scaled,
                                               const int *__restrict__ skip, int TX, int TY, int bx, int by, T *sm) {
    const int w = p + 2;
    const int KX = TX + p + 1, KY = TY + p + 1;   // coarse window I0-p .. I0+TX
    T *es = sm;                                    // [KY][KX]
    T *ts = es + KX * KY;                          // [KY][TX]
    T *rx = ts + KY * TX;                          // [KX][w] rows of the coarse columns
    T *ry = rx + KX * w;                           // [KY][w]
    const int stop = skip ? *skip : 0;
    const int i0 = bx * TX, j0 = by * TY;
    stage_lds<8>(es, KX * KY, [&](int h) {
        const int hx = h % KX, hy = h / KX;
        const int Ix = i0 - p + hx, Iy = j0 - p + hy;
        return (Ix >= 0 && Ix < n1c && Iy >= 0 && Iy < n1c) ? ec[int64_t(Iy) * n1c + Ix] : T(0);
    });
    for (int h = threadIdx.x; h < KX * w; h += blockDim.x) {
        const int I = i0 - p + h / w;
        rx[h] = (I >= 0 && I < n1c) ? R1[int64_t(I) * w + h % w] : T(0);
    }
    for (int h = threadIdx.x; h < KY * w; h += blockDim.x) {
        const int I = j0 - p + h / w;
        ry[h] = (I >= 0 && I < n1c) ? R1[int64_t(I) * w + h % w] : T(0);
    }
    __syncthreads();
    // x pass: ts[row][tx] = sum over the coarse columns kx = tx .. tx+p+1 of
    // R1[kx][tx - kx + p + 1] es[row][kx]  (fine i = i0+tx, coarse I = i0-p+kx)
    for (int h = threadIdx.x; h < KY * TX; h += blockDim.x) {
        const int tx = h % TX, row = h / TX;
        T acc = T(0);
        for (int q = 0; q < w; ++q) {
            const int kx = tx + q;
            acc += rx[kx * w + (p + 1 - q)] * es[row * KX + kx];
        }
        ts[row * TX + tx] = acc;
    }
    __syncthreads();
    if (stop) return;
    // y pass and update, four points per thread at a time: their global
    // operands are loaded before the first is updated
    constexpr int U = 4;
    const int nt = int(blockDim.x);
    for (int base = threadIdx.x; base < TX * TY; base += U * nt) {
        T ov[U];
        double uv[U];
        int64_t gv[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int h = base + u * nt;
            const int tx = h % TX, ty = h / TX;
            const int i = i0 + tx, j = j0 + ty;
            ok[u] = h < TX * TY && i < n1f && j < n1f;
            gv[u] = ok[u] ? int64_t(j) * n1f + i : 0;
            ov[u] = ok[u] ? (mode == 0 ? uf[gv[u]] : e[gv[u]]) : T(0);
            uv[u] = (ok[u] && mode != 0) ? u64[gv[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            const int h = base + u * nt;
            const int tx = h % TX, ty = h / TX;
            T acc = T(0);
            for (int q = 0; q < w; ++q) {
                const int ky = ty + q;
                acc += ry[ky * w + (p + 1 - q)] * ts[ky * TX + tx];
            }
            if (mode == 0) {
                uf[gv[u]] = ov[u] + acc;
            } else {
                const T corr = ov[u] + acc;
                u64[gv[u]] = uv[u] + (scaled ? scal[kScalSigma] * double(corr) : double(corr));
            }
        }
    }
}

template <class T>
__global__ void __launch_bounds__(256) k_prolong2d(const T *__restrict__ R1, int p, int n1f, int n1c,
                                                   const T *__restrict__ ec, T *__restrict__ uf, int mode,
                                                   const T *__restrict__ e, double *__restrict__ u64,
                                                   const double *__restrict__ scal, int scaled,
                                                   const int *__restrict__ skip, int TX, int TY) {
    extern __shared__ unsigned char smem_raw[];
    int bx, by;
    xcd_tile_2d(bx, by);
    prolong2d_body<T>(R1, p, n1f, n1c, ec, uf, mode, e, u64, scal, scaled, skip, TX, TY, bx, by,
                      reinterpret_cast<T *>(smem_raw));
}

// ------------------------------------------------------------------------
// Streamed transfers for large grids (degree-1 coarse space).  As in the
// streamed residual, a workgroup owns a strip of 64 output columns over a
// segment of output rows and walks down it in chunks (here 16 rows, 4 per
// thread); the input rows it needs pass once through an LDS ring of 32 rows,
// the next chunk's rows (and the update's operands) are loaded into registers
// while the current chunk computes, and the two passes of the separable
// transfer are fused per thread: for each input row of its window a thread
// forms the x sum of its column, then adds it with the y weight to each of
// its outputs.  Sums run in the tiled kernels' order.
constexpr int kTrTX = 64, kTrTYT = 4, kTrRY = 4, kTrCH = kTrTYT * kTrRY, kTrRing = 32;
constexpr int kTrTargetGroups = 8192;  // four rounds of eight resident workgroups per CU

// the input window of a streamed transfer: window row q holds input row
// r0 + q at ring slot q % RING, window column hx input column c0 + hx.  Rows
// 0 .. LEAD-1 are staged before the first chunk; chunk c brings rows
// c CH + LEAD .. c CH + LEAD + CH - 1, the strip's 64 columns at window
// columns IX .. IX+63 (row ty + 4u for thread (tx, ty)) and the HX-64 others
// (thread t: row t % CH of halo column t / CH).  Loads read clamped addresses
// unpredicated; positions outside the nin x nin input are zeroed on the way
// into the ring.
template <int HX, int IX, int LEAD, class T>
struct TrWindow {
    static constexpr int TX = kTrTX, CH = kTrCH, RING = kTrRing, NT = kTrTX * kTrTYT;
    static constexpr int NI = CH / kTrTYT, NHC = HX - TX, NH = (NHC * CH + NT - 1) / NT;
    static_assert(CH + LEAD <= RING && (RING & (RING - 1)) == 0, "ring: a power of two holding the window");
    const T *in;
    int nin, r0, c0, tid, tx, ty;
    T xi[NI], xh[NH];
    __device__ int halo_hx(int hc) const { return hc < IX ? hc : TX + hc; }
    __device__ void prefetch(int c) {
        const int rb = r0 + c * CH + LEAD;
        const int cc = min(max(c0 + IX + tx, 0), nin - 1);
#pragma unroll
        for (int u = 0; u < NI; ++u)
            xi[u] = in[int64_t(min(max(rb + ty + kTrTYT * u, 0), nin - 1)) * nin + cc];
#pragma unroll
        for (int u = 0; u < NH; ++u) {
            const int t = tid + u * NT;
            const int gc = c0 + halo_hx(t / CH);
            xh[u] = in[int64_t(min(max(rb + t % CH, 0), nin - 1)) * nin + min(max(gc, 0), nin - 1)];
        }
    }
    __device__ void store(T *ring, int c) const {
        const int q = c * CH + LEAD, rb = r0 + q;
        const int gcol = c0 + IX + tx;
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            const int j = ty + kTrTYT * u, gr = rb + j;
            ring[((q + j) & (RING - 1)) * HX + IX + tx] =
                (gcol >= 0 && gcol < nin && gr >= 0 && gr < nin) ? xi[u] : T(0);
        }
#pragma unroll
        for (int u = 0; u < NH; ++u) {
            const int t = tid + u * NT, j = t % CH, hx = halo_hx(t / CH);
            const int gc = c0 + hx, gr = rb + j;
            if (t < NHC * CH)
                ring[((q + j) & (RING - 1)) * HX + hx] = (gc >= 0 && gc < nin && gr >= 0 && gr < nin) ? xh[u] : T(0);
        }
    }
    __device__ void stage_lead(T *ring) const {
        stage_lds<(LEAD * HX + NT - 1) / NT>(ring, LEAD * HX, [&](int h) {
            const int gc = c0 + h % HX, gr = r0 + h / HX;
            return (gc >= 0 && gc < nin && gr >= 0 && gr < nin) ? in[int64_t(gr) * nin + gc] : T(0);
        });
    }
};

// output rows per segment of a streamed 2-D kernel: whole chunks of ch rows,
// as many segments as bring the launch to about target workgroups (the
// environment variable env, when set, gives another target)
int stream_segment_rows(int64_t n1, int tx, int ch, int64_t target, const char *env) {
    if (const char *e = std::getenv(env)) target = std::max(1L, std::atol(e));
    const int64_t nsx = (n1 + tx - 1) / tx;
    const int64_t nch = (n1 + ch - 1) / ch;
    const int64_t want = std::max<int64_t>(1, target / nsx);
    return int(((nch + want - 1) / want) * ch);
}

// d_c = (R1 (x) R1) d_f: coarse (I, J) takes fine I-1 .. I+P per direction
// with weights R1[I][a], R1[J][b].  Window: fine rows from y0 - 1, fine
// columns from I0 - 1.
template <int P, class T>
__global__ void __launch_bounds__(kTrTX *kTrTYT) k_restrict2d_stream(const T *__restrict__ R1, int n1f, int n1c,
                                                                     int nsx, int nseg, int seg_rows,
                                                                     const T *__restrict__ df, T *__restrict__ dc,
                                                                     const int *__restrict__ skip) {
    constexpr int W = P + 2, HX = kTrTX + P + 1, RY = kTrRY, CH = kTrCH, RING = kTrRing;
    __shared__ T ring[RING * HX];
    if (skip && *skip) return;
    int bx, bs;
    xcd_relabel(int(blockIdx.x), nsx, nsx * nseg, bx, bs);
    const int I0 = bx * kTrTX, y0 = bs * seg_rows, y1 = min(y0 + seg_rows, n1c);
    const int nch = (y1 - y0 + CH - 1) / CH;
    const int tid = int(threadIdx.x), tx = tid % kTrTX;
    const int ty = __builtin_amdgcn_readfirstlane(tid / kTrTX);
    const int I = I0 + tx;
    T rx[W];
#pragma unroll
    for (int a = 0; a < W; ++a) rx[a] = I < n1c ? R1[int64_t(I) * W + a] : T(0);
    TrWindow<HX, 1, P + 1, T> win{df, n1f, y0 - 1, I0 - 1, tid, tx, ty, {}, {}};
    win.stage_lead(ring);
    win.prefetch(0);
    win.store(ring, 0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const bool more = c + 1 < nch;
        if (more) win.prefetch(c + 1);
        const int J0 = y0 + c * CH + ty * RY, q0 = c * CH + ty * RY;
        T acc[RY];
#pragma unroll
        for (int k = 0; k < RY; ++k) acc[k] = T(0);
        if (J0 < y1) {
            T ry[RY][W];
#pragma unroll
            for (int k = 0; k < RY; ++k)
#pragma unroll
                for (int bb = 0; bb < W; ++bb) ry[k][bb] = J0 + k < n1c ? R1[int64_t(J0 + k) * W + bb] : T(0);
#pragma unroll
            for (int yy = 0; yy < RY + W - 1; ++yy) {
                const T *row = ring + ((q0 + yy) & (RING - 1)) * HX + tx;
                T xs = T(0);
#pragma unroll
                for (int a = 0; a < W; ++a) xs += rx[a] * row[a];
#pragma unroll
                for (int k = 0; k < RY; ++k) {
                    const int bb = yy - k;
                    if (bb >= 0 && bb < W) acc[k] += ry[k][bb] * xs;
                }
            }
        }
        if (more) {
            __syncthreads();
            win.store(ring, c + 1);
            __syncthreads();
        }
        if (I < n1c) {
#pragma unroll
            for (int k = 0; k < RY; ++k)
                if (J0 + k < y1) dc[int64_t(J0 + k) * n1c + I] = acc[k];
        }
    }
}

// (R1 (x) R1)^T e_c: fine (i, j) takes coarse I = i-P .. i+1 (and J alike)
// with weight R1[I][i-I+1] R1[J][j-J+1].  MODE 0: uf += P e_c; MODE 1:
// u64 += sigma (e + P e_c) (sigma from scal when scaled, else 1).  Window:
// coarse rows from y0 - P, coarse columns from i0 - P.
template <int P, class T, int MODE>
__global__ void __launch_bounds__(kTrTX *kTrTYT) k_prolong2d_stream(const T *__restrict__ R1, int n1f, int n1c,
                                                                    int nsx, int nseg, int seg_rows,
                                                                    const T *__restrict__ ec, T *__restrict__ uf,
                                                                    const T *__restrict__ e, double *__restrict__ u64,
                                                                    const double *__restrict__ scal, int scaled,
                                                                    const int *__restrict__ skip) {
    constexpr int W = P + 2, HX = kTrTX + P + 1, RY = kTrRY, CH = kTrCH, RING = kTrRing;
    __shared__ T ring[RING * HX];
    if (skip && *skip) return;
    int bx, bs;
    xcd_relabel(int(blockIdx.x), nsx, nsx * nseg, bx, bs);
    const int i0 = bx * kTrTX, y0 = bs * seg_rows, y1 = min(y0 + seg_rows, n1f);
    const int nch = (y1 - y0 + CH - 1) / CH;
    const int tid = int(threadIdx.x), tx = tid % kTrTX;
    const int ty = __builtin_amdgcn_readfirstlane(tid / kTrTX);
    const int i = i0 + tx, ic = min(i, n1f - 1);
    // weight of window column tx + q (coarse I = i - P + q): R1[I][P+1-q]
    T cx[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
        const int Ic = i - P + q;
        cx[q] = (Ic >= 0 && Ic < n1c) ? R1[int64_t(Ic) * W + (P + 1 - q)] : T(0);
    }
    const double sigma = (MODE == 1 && scaled) ? scal[kScalSigma] : 1.0;
    TrWindow<HX, P, P + 1, T> win{ec, n1c, y0 - P, i0 - P, tid, tx, ty, {}, {}};
    // the update's operands at the thread's outputs, double-buffered
    T ov[RY], on[RY];
    double uv[RY], un[RY];
    auto prefetch_out = [&](int c, T *o, double *uu) {
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int64_t g = int64_t(min(y0 + c * CH + ty * RY + k, n1f - 1)) * n1f + ic;
            if constexpr (MODE == 0) {
                o[k] = uf[g];
            } else {
                o[k] = e[g];
                uu[k] = u64[g];
            }
        }
    };
    win.stage_lead(ring);
    prefetch_out(0, ov, uv);
    win.prefetch(0);
    win.store(ring, 0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const bool more = c + 1 < nch;
        if (more) {
            prefetch_out(c + 1, on, un);
            win.prefetch(c + 1);
        }
        const int j0 = y0 + c * CH + ty * RY, q0 = c * CH + ty * RY;
        T acc[RY];
#pragma unroll
        for (int k = 0; k < RY; ++k) acc[k] = T(0);
        if (j0 < y1) {
            T cy[RY][W];
#pragma unroll
            for (int k = 0; k < RY; ++k)
#pragma unroll
                for (int bb = 0; bb < W; ++bb) {
                    const int J = j0 + k - P + bb;
                    cy[k][bb] = (J >= 0 && J < n1c) ? R1[int64_t(J) * W + (P + 1 - bb)] : T(0);
                }
#pragma unroll
            for (int yy = 0; yy < RY + W - 1; ++yy) {
                const T *row = ring + ((q0 + yy) & (RING - 1)) * HX + tx;
                T xs = T(0);
#pragma unroll
                for (int q = 0; q < W; ++q) xs += cx[q] * row[q];
#pragma unroll
                for (int k = 0; k < RY; ++k) {
                    const int bb = yy - k;
                    if (bb >= 0 && bb < W) acc[k] += cy[k][bb] * xs;
                }
            }
        }
        if (more) {
            __syncthreads();
            win.store(ring, c + 1);
            __syncthreads();
        }
        if (i < n1f) {
#pragma unroll
            for (int k = 0; k < RY; ++k) {
                const int j = j0 + k;
                if (j >= y1) continue;
                const int64_t g = int64_t(j) * n1f + i;
                if constexpr (MODE == 0) {
                    uf[g] = ov[k] + acc[k];
                } else {
                    const T corr = ov[k] + acc[k];
                    u64[g] = uv[k] + (scaled ? sigma * double(corr) : double(corr));
                }
            }
        }
        if (more) {
#pragma unroll
            for (int k = 0; k < RY; ++k) {
                ov[k] = on[k];
                if constexpr (MODE == 1) uv[k] = un[k];
            }
        }
    }
}

// ----------------------------------------------------------- batched --
template <class T>
constexpr int prec_slot() { return std::is_same<T, double>::value ? 0 : 1; }

template <class T>
__global__ void __launch_bounds__(256) kb_restrict2d(const BatchProb *__restrict__ bp, const int2 *__restrict__ map,
                                                     int role_f, int role_c) {
    extern __shared__ unsigned char smem_raw[];
    const int2 m = map[blockIdx.x];
    const BatchProb &q = bp[m.x];
    int bx, by;
    xcd_relabel(m.y, q.tr_ntx, q.tr_ntx * q.tr_nty, bx, by);
    restrict2d_body<T>(static_cast<const T *>(q.R1[prec_slot<T>()]), q.p, q.n1, q.n1c,
                       static_cast<const T *>(q.vec[role_f]), static_cast<T *>(q.vec[role_c]), q.flags, q.tr_cx,
                       q.tr_cy, bx, by, reinterpret_cast<T *>(smem_raw));
}

// u64 += sigma (e + P e_c): the end of a correction cycle
template <class T>
__global__ void __launch_bounds__(256) kb_prolong_update2d(const BatchProb *__restrict__ bp,
                                                           const int2 *__restrict__ map, int role_c, int role_e,
                                                           int scaled) {
    extern __shared__ unsigned char smem_raw[];
    const int2 m = map[blockIdx.x];
    const BatchProb &q = bp[m.x];
    int bx, by;
    xcd_relabel(m.y, q.pr_ntx, q.pr_ntx * q.pr_nty, bx, by);
    prolong2d_body<T>(static_cast<const T *>(q.R1[prec_slot<T>()]), q.p, q.n1, q.n1c,
                      static_cast<const T *>(q.vec[role_c]), static_cast<T *>(nullptr), 1,
                      static_cast<const T *>(q.vec[role_e]), static_cast<double *>(q.vec[kVecU]), q.scal, scaled,
                      q.flags, q.pr_tx, q.pr_ty, bx, by, reinterpret_cast<T *>(smem_raw));
}

// the 1-D transfer factor: D1^{-1} Mmix1 (lumped), or Mmix1 when the exact
// transfers apply M_1^{-1} separately
template <class T>
const T *R1_of(const Problem &P) {
    if (P.transfer_exact)
        return std::is_same<T, double>::value ? reinterpret_cast<const T *>(P.Mx64.ptr)
                                              : reinterpret_cast<const T *>(P.Mx32.ptr);
    return std::is_same<T, double>::value ? reinterpret_cast<const T *>(P.R1d64.ptr)
                                          : reinterpret_cast<const T *>(P.R1d32.ptr);
}

template <class T>
const T *fac_of(const Problem &P) {
    return std::is_same<T, double>::value ? reinterpret_cast<const T *>(P.fac64.ptr)
                                          : reinterpret_cast<const T *>(P.fac32.ptr);
}

template <class T>
const T *cf_of(const Problem &P) {
    return std::is_same<T, double>::value ? reinterpret_cast<const T *>(P.cf64.ptr)
                                          : reinterpret_cast<const T *>(P.cf32.ptr);
}

// frame workgroups of the streamed residual: enough for the frame's points,
// rounded up to a multiple of the XCD count
int64_t residual2d_frame_groups(const Problem &Pb) {
    const int64_t n1 = Pb.fine.n1, lr = Pb.ulo + (n1 - 1 - Pb.uhi);
    const int64_t nf = lr * n1 + (Pb.uhi - Pb.ulo + 1) * lr;
    const int64_t g = (nf + kResTX * kResTYT - 1) / (kResTX * kResTYT);
    return (g + kNumXcd - 1) / kNumXcd * kNumXcd;
}

bool residual2d_streamed(const Problem &Pb) {
    return Pb.cf64.ptr != nullptr && Pb.fac64.ptr != nullptr && Pb.uhi >= Pb.ulo;
}

template <int P, class T, bool NORM>
void res2d_launch(const Problem &Pb, const T *val, const T *x, const T *b, T *r, double *partial, hipStream_t s) {
    const int n1 = Pb.fine.n1;
    if (!residual2d_streamed(Pb)) {
        const dim3 grid(nblk(n1, kResTX), nblk(n1, kResCH));
        hipLaunchKernelGGL((k_residual2d_tiled<P, T, NORM>), grid, dim3(kResTX * kResTYT), 0, s, val, Pb.A.npad,
                           Pb.A.pitch[1], n1, x, b, r, partial, Pb.skip);
        return;
    }
    const int seg = residual2d_segment_rows(n1);
    const int nsx = int(nblk(n1, kResTX)), nseg = int(nblk(n1, seg));
    const int nfg = int(residual2d_frame_groups(Pb));
    hipLaunchKernelGGL((k_residual2d<P, T, NORM>), dim3(nfg + nsx * nseg), dim3(kResTX * kResTYT), 0, s,
                       fac_of<T>(Pb), n1, nfg, nsx, nseg, seg, x, b, r, partial, cf_of<T>(Pb), Pb.ulo, Pb.uhi,
                       Pb.skip);
}

template <class T, bool NORM>
void res2d_dispatch(const Problem &Pb, const T *val, const T *x, const T *b, T *r, double *partial, hipStream_t s) {
    switch (Pb.p) {
        case 1: res2d_launch<1, T, NORM>(Pb, val, x, b, r, partial, s); break;
        case 2: res2d_launch<2, T, NORM>(Pb, val, x, b, r, partial, s); break;
        case 3: res2d_launch<3, T, NORM>(Pb, val, x, b, r, partial, s); break;
        case 4: res2d_launch<4, T, NORM>(Pb, val, x, b, r, partial, s); break;
        case 5: res2d_launch<5, T, NORM>(Pb, val, x, b, r, partial, s); break;
        case 6: res2d_launch<6, T, NORM>(Pb, val, x, b, r, partial, s); break;
        case 7: res2d_launch<7, T, NORM>(Pb, val, x, b, r, partial, s); break;
        case 8: res2d_launch<8, T, NORM>(Pb, val, x, b, r, partial, s); break;
        default: throw Error{IGA2L_EUNSUPPORTED, "degree out of range"};
    }
}

}  // namespace

int64_t residual2d_workgroups(const Problem &P) {
    const int64_t n1 = P.fine.n1;
    if (!residual2d_streamed(P)) return ((n1 + kResTX - 1) / kResTX) * ((n1 + kResCH - 1) / kResCH);
    const int64_t seg = residual2d_segment_rows(n1);
    return residual2d_frame_groups(P) + ((n1 + kResTX - 1) / kResTX) * ((n1 + seg - 1) / seg);
}

template <class T>
void launch_residual2d(const Problem &P, const T *val, const T *x, const T *b, T *r, double *partial,
                       hipStream_t s) {
    if (partial) res2d_dispatch<T, true>(P, val, x, b, r, partial, s);
    else res2d_dispatch<T, false>(P, val, x, b, r, nullptr, s);
}
template void launch_residual2d<double>(const Problem &, const double *, const double *, const double *, double *,
                                        double *, hipStream_t);
template void launch_residual2d<float>(const Problem &, const float *, const float *, const float *, float *,
                                       double *, hipStream_t);

namespace {

template <int P, class T>
void restrict2d_stream_launch(const Problem &Pb, const T *df, T *dc, hipStream_t s) {
    const int n1c = Pb.coarse.n1;
    const int seg = stream_segment_rows(n1c, kTrTX, kTrCH, kTrTargetGroups, "IGA2L_TRANSFER_GROUPS");
    const int nsx = int(nblk(n1c, kTrTX)), nseg = int(nblk(n1c, seg));
    hipLaunchKernelGGL((k_restrict2d_stream<P, T>), dim3(nsx * nseg), dim3(kTrTX * kTrTYT), 0, s, R1_of<T>(Pb),
                       Pb.fine.n1, n1c, nsx, nseg, seg, df, dc, Pb.skip);
}

template <int P, class T>
void prolong2d_stream_launch(const Problem &Pb, const T *ec, T *uf, const T *e, double *u64, bool scaled,
                             hipStream_t s) {
    const int n1f = Pb.fine.n1;
    const int seg = stream_segment_rows(n1f, kTrTX, kTrCH, kTrTargetGroups, "IGA2L_TRANSFER_GROUPS");
    const int nsx = int(nblk(n1f, kTrTX)), nseg = int(nblk(n1f, seg));
    if (u64)
        hipLaunchKernelGGL((k_prolong2d_stream<P, T, 1>), dim3(nsx * nseg), dim3(kTrTX * kTrTYT), 0, s,
                           R1_of<T>(Pb), n1f, Pb.coarse.n1, nsx, nseg, seg, ec, static_cast<T *>(nullptr), e, u64,
                           Pb.scal.as<double>(), scaled ? 1 : 0, Pb.skip);
    else
        hipLaunchKernelGGL((k_prolong2d_stream<P, T, 0>), dim3(nsx * nseg), dim3(kTrTX * kTrTYT), 0, s,
                           R1_of<T>(Pb), n1f, Pb.coarse.n1, nsx, nseg, seg, ec, uf, static_cast<const T *>(nullptr),
                           static_cast<double *>(nullptr), static_cast<const double *>(nullptr), 0, Pb.skip);
}

// the streamed transfers serve grids of at least 2^20 fine points
bool transfer2d_streamed(const Problem &P) { return P.plow == 1 && P.fine.n >= (int64_t(1) << 20); }

}  // namespace

#define IGA2L_TR_DISPATCH(F, ...)                                        \
    switch (P.p) {                                                       \
        case 1: F<1, T>(__VA_ARGS__); break;                             \
        case 2: F<2, T>(__VA_ARGS__); break;                             \
        case 3: F<3, T>(__VA_ARGS__); break;                             \
        case 4: F<4, T>(__VA_ARGS__); break;                             \
        case 5: F<5, T>(__VA_ARGS__); break;                             \
        case 6: F<6, T>(__VA_ARGS__); break;                             \
        case 7: F<7, T>(__VA_ARGS__); break;                             \
        case 8: F<8, T>(__VA_ARGS__); break;                             \
        default: throw Error{IGA2L_EUNSUPPORTED, "degree out of range"}; \
    }

template <class T>
void launch_restrict2d(const Problem &P, const T *df, T *dc, hipStream_t s) {
    if (transfer2d_streamed(P)) {
        IGA2L_TR_DISPATCH(restrict2d_stream_launch, P, df, dc, s);
        return;
    }
    const int p = P.p;
    int CX, CY;
    transfer_tile_2d(P.coarse.n1, CX, CY);
    const size_t shm = restrict2d_lds(p, CX, CY, sizeof(T));
    const dim3 grid(nblk(P.coarse.n1, CX), nblk(P.coarse.n1, CY));
    hipLaunchKernelGGL((k_restrict2d<T>), grid, dim3(256), shm, s, R1_of<T>(P), p, P.fine.n1, P.coarse.n1, df, dc,
                       P.skip, CX, CY);
}
template void launch_restrict2d<double>(const Problem &, const double *, double *, hipStream_t);
template void launch_restrict2d<float>(const Problem &, const float *, float *, hipStream_t);

template <class T>
void launch_prolong2d(const Problem &P, const T *ec, T *uf, const T *e, double *u64, bool scaled, hipStream_t s) {
    if (transfer2d_streamed(P)) {
        IGA2L_TR_DISPATCH(prolong2d_stream_launch, P, ec, uf, e, u64, scaled, s);
        return;
    }
    const int p = P.p;
    int TX, TY;
    transfer_tile_2d(P.fine.n1, TX, TY);
    const size_t shm = prolong2d_lds(p, TX, TY, sizeof(T));
    const dim3 grid(nblk(P.fine.n1, TX), nblk(P.fine.n1, TY));
    hipLaunchKernelGGL((k_prolong2d<T>), grid, dim3(256), shm, s, R1_of<T>(P), p, P.fine.n1, P.coarse.n1, ec, uf,
                       u64 ? 1 : 0, e, u64, P.scal.as<double>(), scaled ? 1 : 0, P.skip, TX, TY);
}
template void launch_prolong2d<double>(const Problem &, const double *, double *, const double *, double *, bool,
                                       hipStream_t);
template void launch_prolong2d<float>(const Problem &, const float *, float *, const float *, double *, bool,
                                      hipStream_t);

#undef IGA2L_TR_DISPATCH

size_t restrict2d_lds(int p, int cx, int cy, size_t elem) {
    const size_t w = p + 2, FX = cx + p + 1, FY = cy + p + 1;
    return (FX * FY + FY * cx + cx * w + cy * w) * elem;
}

size_t prolong2d_lds(int p, int tx, int ty, size_t elem) {
    const size_t w = p + 2, KX = tx + p + 1, KY = ty + p + 1;
    return (KX * KY + KY * tx + KX * w + KY * w) * elem;
}

template <class T>
void launch_restrict_batch(const BatchProb *bp, const int2 *map, int nwg, size_t shm, int role_f, int role_c,
                           hipStream_t s) {
    hipLaunchKernelGGL((kb_restrict2d<T>), dim3(nwg), dim3(256), shm, s, bp, map, role_f, role_c);
}
template void launch_restrict_batch<double>(const BatchProb *, const int2 *, int, size_t, int, int, hipStream_t);
template void launch_restrict_batch<float>(const BatchProb *, const int2 *, int, size_t, int, int, hipStream_t);

template <class T>
void launch_prolong_update_batch(const BatchProb *bp, const int2 *map, int nwg, size_t shm, int role_c, int role_e,
                                 bool scaled, hipStream_t s) {
    hipLaunchKernelGGL((kb_prolong_update2d<T>), dim3(nwg), dim3(256), shm, s, bp, map, role_c, role_e,
                       scaled ? 1 : 0);
}
template void launch_prolong_update_batch<double>(const BatchProb *, const int2 *, int, size_t, int, int, bool,
                                                  hipStream_t);
template void launch_prolong_update_batch<float>(const BatchProb *, const int2 *, int, size_t, int, int, bool,
                                                 hipStream_t);

}  // namespace iga2l
