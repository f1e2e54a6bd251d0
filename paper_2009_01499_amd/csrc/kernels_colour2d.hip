// kernels_colour2d.hip -- one colour of the multiplicative Schwarz sweep
// (Section 3, the coloured variant with colour period s = b) on large 2-D
// grids with kappa = 1, streamed through HBM like the 2-D residual.
//
// With s = b every point lies in exactly one b x b block of the colour, so a
// colour is: r = f - A x on every point, then x += A_blk^{-1} r_blk per block.
// A workgroup owns a strip of whole cells (63 or 60 columns) and a segment of
// rows; it walks the segment in chunks of four thread rows of one to three
// cell rows each (more for 3 x 3 blocks: fewer window rows per output).  The
// x rows of a chunk's window sit in an LDS ring, the next chunk's rows (and
// right-hand side) are loaded into registers while the current chunk
// computes, the residual of the chunk's cells goes to LDS, and each point
// then applies its row of its block's inverse.  Interior rows apply
// A = K1 (x) M1 + M1 (x) K1 by sum factorisation from the interior 1-D rows
// (symmetric: the x sums add the two entries that share a weight first);
// wavefronts that touch the frame of points within ulo of the boundary take
// every 1-D row from the factors.  The interior blocks' shared inverse is
// staged in LDS (b <= 5).  With the default workgroup target every segment
// is one chunk on large grids (more workgroups in flight measured faster
// than longer streams), which an instance without the prefetch registers
// serves; the first colour of a sweep from a zero iterate has a kernel of
// its own (no halo).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "internal.h"

namespace iga2l {

namespace {

constexpr int kCsTXT = 64, kCsTYT = 4, kCsNT = kCsTXT * kCsTYT;
constexpr int kCsTargetGroups = 16384;
// cell rows per thread: for 3 x 3 blocks two (FP64) or three (FP32, whose
// registers are half the size) where the chunk window fits a 32- or 64-row
// ring (fewer window rows per output), one otherwise
template <int P, int B, class T>
constexpr int kCellRows = (B != 3) ? 1
                          : (sizeof(T) == 4 && kCsTYT * 3 * B + 2 * P <= 64) ? 3
                          : (kCsTYT * 2 * B + 2 * P <= 32) ? 2 : 1;

// ONE: every segment is a single chunk (the launch shape of large grids
// with the default workgroup target), so no rows are prefetched and the
// registers that would hold them go to occupancy
template <int P, int B, class T, bool ONE>
__global__ void __launch_bounds__(kCsNT, (ONE && B == 3) ? 5 : 1)
    k_colour2d_stream(const T *__restrict__ fac, const T *__restrict__ cf, int n1, int ulo, int uhi,
                      const T *__restrict__ inv, int clsL, int ncls1, const T *__restrict__ x_src,
                      T *__restrict__ x_dst, const T *__restrict__ rhs, int ox, int oy, int nsx, int nseg,
                      int seg_rows, const int *__restrict__ skip) {
    constexpr int TX = (kCsTXT / B) * B;  // strip columns: whole cells
    constexpr int RY = kCellRows<P, B, T> * B;  // rows per thread: whole cell rows
    constexpr int CH = kCsTYT * RY;          // chunk rows
    constexpr int HX = TX + 2 * P;
    constexpr int W1 = 2 * P + 1, BD = B * B, HB = (B - 1) / 2;
    // a single chunk's window exactly, else a power of two holding one
    constexpr int RING = ONE ? CH + 2 * P : (CH + 2 * P <= 32) ? 32 : 64;
    constexpr bool kLdsInv = BD * BD * sizeof(T) <= 8192;
    static_assert(CH + 2 * P <= RING, "ring holds the window");
    __shared__ T ring[RING * HX];
    // ring slot of window row q (the single-chunk window does not wrap)
    auto slot = [](int q) { return ONE ? q : (q & (RING - 1)); };
    __shared__ T rs[CH * TX];
    __shared__ T ivs[kLdsInv ? BD * BD : 1];
    if (skip && *skip) return;
    int bx, bs;
    xcd_relabel(int(blockIdx.x), nsx, nsx * nseg, bx, bs);
    const int gx0 = ox + bx * TX, y0 = oy + bs * seg_rows;
    const int y1 = min(y0 + seg_rows, n1);
    const int nch = ONE ? 1 : (y1 - y0 + CH - 1) / CH;
    const int tid = int(threadIdx.x);
    const int tx = tid % kCsTXT;
    // the thread row is the wavefront's: rows and their 1-D factors are uniform
    const int ty = __builtin_amdgcn_readfirstlane(tid / kCsTXT);
    const bool act = tx < TX;
    const int gx = gx0 + tx;
    const bool col_in = act && gx >= 0 && gx < n1;
    const int gxc = min(max(gx, 0), n1 - 1);
    const int64_t nw = int64_t(n1) * W1;
    if constexpr (kLdsInv) {
        const int64_t islot = int64_t(clsL) + int64_t(ncls1) * clsL;
        for (int h = tid; h < BD * BD; h += kCsNT) ivs[h] = inv[islot * BD * BD + h];
    }
    // window row q (0-based from global row y0 - P) sits in ring slot q % RING,
    // window column hx at global column gx0 - P + hx; the 2P rows above the
    // first chunk first
    stage_lds<(2 * P * HX + kCsNT - 1) / kCsNT>(ring, 2 * P * HX, [&](int h) {
        const int hgx = gx0 + h % HX - P, hgy = y0 - P + h / HX;
        return (hgx >= 0 && hgx < n1 && hgy >= 0 && hgy < n1) ? x_src[int64_t(hgy) * n1 + hgx] : T(0);
    });
    // chunk c's new rows (global rows y0 + c CH + P + j): the strip columns,
    // row ty + 4u for thread (tx, ty), and the 2P halo columns, thread t taking
    // row t % CH of halo column t / CH.  Clamped addresses, unpredicated loads;
    // positions outside the grid are zeroed where the values enter the ring.
    constexpr int NI = CH / kCsTYT, NH = (2 * P * CH + kCsNT - 1) / kCsNT;
    T xi[NI], xh[NH];
    auto halo_col = [&](int hc) { return hc < P ? gx0 - P + hc : gx0 + TX - P + hc; };
    auto clampy = [&](int y) { return min(max(y, 0), n1 - 1); };
    auto prefetch = [&](int c) {
        const int ybase = y0 + c * CH + P;
#pragma unroll
        for (int u = 0; u < NI; ++u) xi[u] = x_src[int64_t(clampy(ybase + ty + kCsTYT * u)) * n1 + gxc];
#pragma unroll
        for (int u = 0; u < NH; ++u) {
            const int t = tid + u * kCsNT;
            const int gxh = halo_col(t / CH);
            xh[u] = x_src[int64_t(clampy(ybase + t % CH)) * n1 + min(max(gxh, 0), n1 - 1)];
        }
    };
    auto store_ring = [&](int c) {
        const int q = c * CH + 2 * P, ybase = y0 + c * CH + P;
        if (act) {
#pragma unroll
            for (int u = 0; u < NI; ++u) {
                const int j = ty + kCsTYT * u, y = ybase + j;
                ring[slot(q + j) * HX + P + tx] = (col_in && y >= 0 && y < n1) ? xi[u] : T(0);
            }
        }
#pragma unroll
        for (int u = 0; u < NH; ++u) {
            const int t = tid + u * kCsNT, j = t % CH, hc = t / CH;
            const int gxh = halo_col(hc), y = ybase + j;
            if (t < 2 * P * CH)
                ring[slot(q + j) * HX + (hc < P ? hc : TX + hc)] =
                    (gxh >= 0 && gxh < n1 && y >= 0 && y < n1) ? xh[u] : T(0);
        }
    };
    // the right-hand side of the thread's RY rows
    T bv[RY], bn[RY];
    auto prefetch_b = [&](int c, T *dst) {
#pragma unroll
        for (int k = 0; k < RY; ++k) dst[k] = rhs[int64_t(clampy(y0 + c * CH + ty * RY + k)) * n1 + gxc];
    };
    prefetch_b(0, bv);
    prefetch(0);
    store_ring(0);
    __syncthreads();
    // the strip's columns carry the interior 1-D rows (wavefront-uniform)
    const bool cols_uni = __all(!act || (gx >= ulo && gx <= uhi));
    const T *Kx = fac + int64_t(gxc) * W1, *Mx = fac + nw + int64_t(gxc) * W1;
    // the point's place in its block and the block's cell in the strip
    const int cx = tx % B, cell0 = (tx / B) * B;
    const int ccx = gx0 + cell0 + HB;
    const int clx = (ccx >= 0 && ccx < n1) ? block_class(ccx, n1, clsL) : -1;
    for (int c = 0; c < nch; ++c) {
        const bool more = c + 1 < nch;
        if (more) {
            prefetch_b(c + 1, bn);
            prefetch(c + 1);
        }
        const int gyb = y0 + c * CH + ty * RY;  // the thread's first row
        const int q0 = c * CH + ty * RY;        // its window row, minus P
        T acc[RY], xc[RY];
#pragma unroll
        for (int k = 0; k < RY; ++k) acc[k] = xc[k] = T(0);
        // (cell rows past the segment have nothing to compute; keeping the
        // arithmetic under this chunk-dependent test also keeps the compiler
        // from holding the unrolled window in registers)
        if (act && gyb < y1) {
            const bool rows_uni = gyb >= ulo && gyb + RY - 1 <= uhi;
            if (cols_uni && rows_uni) {
                // row yy of the window (0 .. RY+2P-1) feeds output k with oy = yy - k;
                // the interior rows are symmetric (checked on the host), so
                // the x sums pair the entries o and 2P - o
#pragma unroll
                for (int yy = 0; yy < RY + 2 * P; ++yy) {
                    const T *row = ring + slot(q0 + yy) * HX + tx;
                    T kx = cf[P] * row[P], mx = cf[W1 + P] * row[P];
#pragma unroll
                    for (int o = 0; o < P; ++o) {
                        const T v = row[o] + row[2 * P - o];
                        kx += cf[o] * v;
                        mx += cf[W1 + o] * v;
                    }
#pragma unroll
                    for (int k = 0; k < RY; ++k) {
                        const int oy = yy - k;
                        if (oy >= 0 && oy < W1) {
                            // two fused multiply-adds into the accumulator
                            acc[k] += cf[oy] * mx;
                            acc[k] += cf[W1 + oy] * kx;
                        }
                    }
                }
            } else {
                // the frame: every 1-D row from the factors (entries that
                // would leave the grid are zero there)
#pragma unroll 1
                for (int yy = 0; yy < RY + 2 * P; ++yy) {
                    const T *row = ring + slot(q0 + yy) * HX + tx;
                    T mx = T(0), kx = T(0);
#pragma unroll
                    for (int o = 0; o < W1; ++o) {
                        const T v = row[o];
                        kx += Kx[o] * v;
                        mx += Mx[o] * v;
                    }
#pragma unroll
                    for (int k = 0; k < RY; ++k) {
                        const int oy = yy - k;
                        if (oy >= 0 && oy < W1) {
                            const int64_t fy = int64_t(clampy(gyb + k)) * W1 + oy;
                            acc[k] += fac[fy] * mx + fac[nw + fy] * kx;
                        }
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < RY; ++k) xc[k] = ring[slot(q0 + P + k) * HX + P + tx];
        }
        __syncthreads();  // the ring rows and the residuals of the last chunk are read
        if (act) {
#pragma unroll
            for (int k = 0; k < RY; ++k) {
                const int gy = gyb + k;
                rs[(ty * RY + k) * TX + tx] = (col_in && gy >= 0 && gy < n1) ? bv[k] - acc[k] : T(0);
            }
        }
        if (more) store_ring(c + 1);
        __syncthreads();
        // x += (row of the block's inverse) . (the block's residuals), per cell
        // row: its residuals read once, then one inverse row per output
        if (col_in && gyb < y1) {
#pragma unroll
            for (int j = 0; j < RY / B; ++j) {
                const int cb = gyb + j * B;  // the cell's first row
                const int ccy = cb + HB;
                const T *rblk = rs + (ty * RY + j * B) * TX + cell0;
                T rv[BD], delta[B];
#pragma unroll
                for (int l = 0; l < BD; ++l) rv[l] = rblk[(l / B) * TX + l % B];
#pragma unroll
                for (int kk = 0; kk < B; ++kk) delta[kk] = T(0);
                if (clx >= 0 && ccy >= 0 && ccy < n1) {
                    const int cly = block_class(ccy, n1, clsL);
                    if (kLdsInv && clx == clsL && cly == clsL) {
                        const T *irow = ivs + cx * BD;
#pragma unroll
                        for (int kk = 0; kk < B; ++kk)
#pragma unroll
                            for (int l = 0; l < BD; ++l) delta[kk] += irow[kk * B * BD + l] * rv[l];
                    } else {
                        const T *irow = inv + ((int64_t(clx) + int64_t(ncls1) * cly) * BD + cx) * BD;
#pragma unroll
                        for (int kk = 0; kk < B; ++kk)
#pragma unroll
                            for (int l = 0; l < BD; ++l) delta[kk] += irow[kk * B * BD + l] * rv[l];
                    }
                }
#pragma unroll
                for (int kk = 0; kk < B; ++kk) {
                    const int gy = cb + kk;
                    if (gy >= 0 && gy < y1) x_dst[int64_t(gy) * n1 + gx] = xc[j * B + kk] + delta[kk];
                }
            }
        }
        if (more) {
#pragma unroll
            for (int k = 0; k < RY; ++k) bv[k] = bn[k];
        }
    }
}

// cell rows per thread of the zero-start colour: two for 3 x 3 blocks (more
// loads in flight per thread), one otherwise
template <int B>
constexpr int kZeroCellRows = (B == 3) ? 2 : 1;

// The first colour of a sweep from a zero iterate (x_zero): the residual is
// the right-hand side itself (or r64 / sigma, cast to T and stored to rhs_out
// for the later colours), so a workgroup needs no halo: a tile of whole cells
// (the strip width by four thread rows of whole cell rows) loads its residuals
// to LDS and applies the block inverses, x = A_blk^{-1} r_blk.  The block
// solve is the streamed colour's, in the same summation order.
template <int B, class T>
__global__ void __launch_bounds__(kCsNT)
    k_colour2d_zero(const T *__restrict__ inv, int clsL, int ncls1, int n1, const T *__restrict__ rhs,
                    const double *__restrict__ r64, const double *__restrict__ scal, T *__restrict__ rhs_out,
                    T *__restrict__ x_dst, int ox, int oy, int nsx, int nty, const int *__restrict__ skip) {
    constexpr int TX = (kCsTXT / B) * B, RY = kZeroCellRows<B> * B, CH = kCsTYT * RY, BD = B * B, HB = (B - 1) / 2;
    constexpr bool kLdsInv = BD * BD * sizeof(T) <= 8192;
    __shared__ T rs[CH * TX];
    __shared__ T ivs[kLdsInv ? BD * BD : 1];
    if (skip && *skip) return;
    int bx, by;
    xcd_relabel(int(blockIdx.x), nsx, nsx * nty, bx, by);
    const int gx0 = ox + bx * TX;
    const int tid = int(threadIdx.x), tx = tid % kCsTXT;
    const int ty = __builtin_amdgcn_readfirstlane(tid / kCsTXT);
    const int gyb = oy + by * CH + ty * RY;  // the thread's first cell row
    const bool act = tx < TX;
    const int gx = gx0 + tx;
    const bool col_in = act && gx >= 0 && gx < n1;
    if constexpr (kLdsInv) {
        const int64_t islot = int64_t(clsL) + int64_t(ncls1) * clsL;
        for (int h = tid; h < BD * BD; h += kCsNT) ivs[h] = inv[islot * BD * BD + h];
    }
    if (act) {
        const double inv_sigma = r64 ? scal[kScalInvSigma] : 1.0;
#pragma unroll
        for (int k = 0; k < RY; ++k) {
            const int gy = gyb + k;
            T v = T(0);
            if (col_in && gy >= 0 && gy < n1) {
                const int64_t gi = int64_t(gy) * n1 + gx;
                if (r64) {
                    v = T(r64[gi] * inv_sigma);
                    rhs_out[gi] = v;
                } else {
                    v = rhs[gi];
                }
            }
            rs[(ty * RY + k) * TX + tx] = v;
        }
    }
    __syncthreads();
    if (!col_in || gyb >= n1) return;
    const int cx = tx % B, cell0 = (tx / B) * B;
    const int ccx = gx0 + cell0 + HB;
#pragma unroll
    for (int j = 0; j < RY / B; ++j) {
        const int cb = gyb + j * B, ccy = cb + HB;  // the cell's first row and centre
        const T *rblk = rs + (ty * RY + j * B) * TX + cell0;
        T rv[BD], delta[B];
#pragma unroll
        for (int l = 0; l < BD; ++l) rv[l] = rblk[(l / B) * TX + l % B];
#pragma unroll
        for (int kk = 0; kk < B; ++kk) delta[kk] = T(0);
        if (ccx >= 0 && ccx < n1 && ccy >= 0 && ccy < n1) {
            const int clx = block_class(ccx, n1, clsL), cly = block_class(ccy, n1, clsL);
            if (kLdsInv && clx == clsL && cly == clsL) {
                const T *irow = ivs + cx * BD;
#pragma unroll
                for (int kk = 0; kk < B; ++kk)
#pragma unroll
                    for (int l = 0; l < BD; ++l) delta[kk] += irow[kk * B * BD + l] * rv[l];
            } else {
                const T *irow = inv + ((int64_t(clx) + int64_t(ncls1) * cly) * BD + cx) * BD;
#pragma unroll
                for (int kk = 0; kk < B; ++kk)
#pragma unroll
                    for (int l = 0; l < BD; ++l) delta[kk] += irow[kk * B * BD + l] * rv[l];
            }
        }
#pragma unroll
        for (int kk = 0; kk < B; ++kk) {
            const int gy = cb + kk;
            if (gy >= 0 && gy < n1) x_dst[int64_t(gy) * n1 + gx] = delta[kk];
        }
    }
}

int colour2d_segment_rows(int64_t n1, int tx, int ch) {
    int64_t target = kCsTargetGroups;
    // IGA2L_COLOUR_GROUPS sets another workgroup target (tests use a small one
    // to send many chunks through each ring)
    if (const char *e = std::getenv("IGA2L_COLOUR_GROUPS")) target = std::max(1L, std::atol(e));
    const int64_t nsx = (n1 + tx - 1) / tx;
    const int64_t nch = (n1 + ch - 1) / ch;
    const int64_t want = std::max<int64_t>(1, target / nsx);
    return int(((nch + want - 1) / want) * ch);
}

template <int P, int B, class T>
void colour2d_stream_launch(const Problem &Pb, int cx, int cy, const T *x_src, T *x_dst, const T *rhs,
                            hipStream_t s) {
    constexpr int TX = (kCsTXT / B) * B, CH = kCsTYT * kCellRows<P, B, T> * B, HB = (B - 1) / 2;
    const int n1 = Pb.fine.n1;
    // strip and segment origins: aligned with the colour's blocks, at or before 0
    int ox = cx - HB, oy = cy - HB;
    if (ox > 0) ox -= B;
    if (oy > 0) oy -= B;
    const int seg_rows = colour2d_segment_rows(n1, TX, CH);
    const int nsx = (n1 - ox + TX - 1) / TX, nseg = (n1 - oy + seg_rows - 1) / seg_rows;
    auto kern = seg_rows == CH ? k_colour2d_stream<P, B, T, true> : k_colour2d_stream<P, B, T, false>;
    constexpr bool f64 = std::is_same<T, double>::value;
    const T *fac = reinterpret_cast<const T *>(f64 ? Pb.fac64.ptr : Pb.fac32.ptr);
    const T *cf = reinterpret_cast<const T *>(f64 ? Pb.cf64.ptr : Pb.cf32.ptr);
    const T *inv = reinterpret_cast<const T *>(f64 ? Pb.Inv64.ptr : Pb.Inv32.ptr);
    hipLaunchKernelGGL(kern, dim3(nsx * nseg), dim3(kCsNT), 0, s, fac, cf, n1, Pb.ulo, Pb.uhi,
                       inv, class_split(Pb), Pb.ncls1, x_src, x_dst, rhs, ox, oy, nsx, nseg, seg_rows, Pb.skip);
}

template <int B, class T>
void colour2d_zero_launch(const Problem &Pb, int cx, int cy, const T *rhs, const double *r64, T *rhs_out, T *x_dst,
                          hipStream_t s) {
    constexpr int TX = (kCsTXT / B) * B, CH = kCsTYT * kZeroCellRows<B> * B, HB = (B - 1) / 2;
    const int n1 = Pb.fine.n1;
    int ox = cx - HB, oy = cy - HB;
    if (ox > 0) ox -= B;
    if (oy > 0) oy -= B;
    const int nsx = (n1 - ox + TX - 1) / TX, nty = (n1 - oy + CH - 1) / CH;
    constexpr bool f64 = std::is_same<T, double>::value;
    const T *inv = reinterpret_cast<const T *>(f64 ? Pb.Inv64.ptr : Pb.Inv32.ptr);
    hipLaunchKernelGGL((k_colour2d_zero<B, T>), dim3(nsx * nty), dim3(kCsNT), 0, s, inv, class_split(Pb), Pb.ncls1, n1,
                       rhs, r64, Pb.scal.as<double>(), rhs_out, x_dst, ox, oy, nsx, nty, Pb.skip);
}

template <class T>
void colour2d_zero_b(const Problem &Pb, int cx, int cy, const T *rhs, const double *r64, T *rhs_out, T *x_dst,
                     hipStream_t s) {
    switch (Pb.bw) {
        case 3: colour2d_zero_launch<3, T>(Pb, cx, cy, rhs, r64, rhs_out, x_dst, s); break;
        case 5: colour2d_zero_launch<5, T>(Pb, cx, cy, rhs, r64, rhs_out, x_dst, s); break;
        default: colour2d_zero_launch<7, T>(Pb, cx, cy, rhs, r64, rhs_out, x_dst, s); break;
    }
}

template <int P, class T>
void colour2d_stream_b(const Problem &Pb, int cx, int cy, const T *x_src, T *x_dst, const T *rhs, hipStream_t s) {
    switch (Pb.bw) {
        case 3: colour2d_stream_launch<P, 3, T>(Pb, cx, cy, x_src, x_dst, rhs, s); break;
        case 5: colour2d_stream_launch<P, 5, T>(Pb, cx, cy, x_src, x_dst, rhs, s); break;
        default: colour2d_stream_launch<P, 7, T>(Pb, cx, cy, x_src, x_dst, rhs, s); break;
    }
}

template <class T>
void colour2d_stream_p(const Problem &Pb, int cx, int cy, const T *x_src, T *x_dst, const T *rhs, hipStream_t s) {
    switch (Pb.p) {
        case 1: colour2d_stream_b<1, T>(Pb, cx, cy, x_src, x_dst, rhs, s); break;
        case 2: colour2d_stream_b<2, T>(Pb, cx, cy, x_src, x_dst, rhs, s); break;
        case 3: colour2d_stream_b<3, T>(Pb, cx, cy, x_src, x_dst, rhs, s); break;
        case 4: colour2d_stream_b<4, T>(Pb, cx, cy, x_src, x_dst, rhs, s); break;
        case 5: colour2d_stream_b<5, T>(Pb, cx, cy, x_src, x_dst, rhs, s); break;
        case 6: colour2d_stream_b<6, T>(Pb, cx, cy, x_src, x_dst, rhs, s); break;
        case 7: colour2d_stream_b<7, T>(Pb, cx, cy, x_src, x_dst, rhs, s); break;
        default: colour2d_stream_b<8, T>(Pb, cx, cy, x_src, x_dst, rhs, s); break;
    }
}

}  // namespace

bool colour2d_stream_ok(const Problem &P, int S) {
    // IGA2L_COLOUR_STREAM=0 in the environment keeps the tiled kernel (read at
    // every launch, so that tests can compare the two in one process)
    const char *v = std::getenv("IGA2L_COLOUR_STREAM");
    if ((v && v[0] == '0') || P.dim != 2 || P.geometry != kGeomSquare || P.fine.n < (int64_t(1) << 19)) return false;
    if (!(P.bw == 3 || P.bw == 5 || P.bw == 7) || S != P.bw || P.p < 1 || P.p > 8) return false;
    if (P.cf64.ptr == nullptr || P.fac64.ptr == nullptr || P.uhi < P.ulo || class_split(P) < 0) return false;
    // the interior rows pair their entries o and 2p - o
    const int w1 = 2 * P.p + 1;
    const size_t ic = size_t(P.fine.n1 / 2) * w1;
    for (int o = 0; o < P.p; ++o)
        if (P.K1[ic + o] != P.K1[ic + 2 * P.p - o] || P.M1[ic + o] != P.M1[ic + 2 * P.p - o]) return false;
    return true;
}

bool colour2d_stream(const Problem &P, int cx, int cy, int S, const void *x_src, void *x_dst, const void *rhs,
                     bool x_zero, const double *r64, void *rhs_out, bool fp64, hipStream_t s) {
    if (!colour2d_stream_ok(P, S)) return false;
    if (x_zero) {
        if (fp64)
            colour2d_zero_b<double>(P, cx, cy, static_cast<const double *>(rhs), r64, static_cast<double *>(rhs_out),
                                    static_cast<double *>(x_dst), s);
        else
            colour2d_zero_b<float>(P, cx, cy, static_cast<const float *>(rhs), r64, static_cast<float *>(rhs_out),
                                   static_cast<float *>(x_dst), s);
        return true;
    }
    if (r64) return false;
    if (fp64)
        colour2d_stream_p<double>(P, cx, cy, static_cast<const double *>(x_src), static_cast<double *>(x_dst),
                                  static_cast<const double *>(rhs), s);
    else
        colour2d_stream_p<float>(P, cx, cy, static_cast<const float *>(x_src), static_cast<float *>(x_dst),
                                 static_cast<const float *>(rhs), s);
    return true;
}

}  // namespace iga2l
