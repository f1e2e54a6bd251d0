// kernels_3d.hip -- 3-D kernels of the two-level solver for kappa = 1 by sum
// factorisation, with the shared Schwarz block inverse applied on the matrix
// cores.
//
// With kappa = 1 the 3-D stiffness matrix is a sum of Kronecker products of
// the 1-D stiffness and mass matrices of the degree-p space (Section 2, the
// tensor-product spline space):  A = Kz My Mx + Mz Ky Mx + Mz My Kx.  On a
// tile held in LDS, A x is three passes of 1-D products with 2p+1 taps:
//   along x:  tM = Mx x,  tK = Kx x;
//   along y:  a = My tM,  b = Ky tM + My tK;
//   along z:  A x = Kz a + Mz b,
// 7 (2p+1)-tap products per point (98 flops at p = 3) instead of the
// (2p+1)^3 = 343 taps of an assembled row.  The factor rows of a point are the
// rows of the 1-D matrices at its coordinates, so rows next to the boundary
// need no special case.
//
// One colour of the coloured Schwarz sweep with 3x3x3 blocks and colour
// period 3 (Section 3.1.1): the blocks of a colour tile the grid, so the
// residual of every point of a tile is needed.  Blocks whose centre lies in
// the interior class in every direction share one 27x27 inverse: their
// corrections are one dense product delta[27 x nb] = Inv[27 x 27] R[27 x nb]
// over the tile's blocks, done with 16x16x4 MFMA instructions (M and K padded
// to 32 and 28, the blocks of the tile in groups of 16).  Blocks next to the
// boundary apply their own class inverse on the vector units.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace iga2l {

namespace {

constexpr int kSfThreads = 512;
constexpr int kSfWaves = kSfThreads / 64;

typedef float sf_f4 __attribute__((ext_vector_type(4)));
typedef double sf_d4 __attribute__((ext_vector_type(4)));

// Tile geometry and LDS layout (in elements of the working precision).
template <int P>
struct Sf {
    static constexpr int TX = 12, TY = 12, TZ = 6;       // whole 3x3x3 blocks
    static constexpr int W1 = 2 * P + 1;
    static constexpr int HX = TX + 2 * P, HY = TY + 2 * P, HZ = TZ + 2 * P;
    static constexpr int NU = HX * HY * HZ;   // iterate over the tile and a halo of width p
    static constexpr int NT = TX * HY * HZ;   // each of tM, tK
    static constexpr int NA = TX * TY * HZ;   // each of a, b
    static constexpr int NR = TX * TY * TZ;   // tile points
    static constexpr bool kReuse = 2 * NA <= NU;   // a, b overwrite the iterate (dead after the x pass)
    static constexpr int OFF_T = NU;                // tM, then tK; later r (residual) and delta
    static constexpr int OFF_A = kReuse ? 0 : NU + 2 * NT;
    static constexpr int OFF_F = kReuse ? NU + 2 * NT : NU + 2 * NT + 2 * NA;   // factor rows
    static constexpr int NF = (TX + TY + TZ) * 2 * W1;
    static constexpr int LDS = OFF_F + NF;
    static constexpr int OFF_R = OFF_T, OFF_D = OFF_T + NT;
    static constexpr int NBX = TX / 3, NBY = TY / 3, NBZ = TZ / 3, NB = NBX * NBY * NBZ;
    static constexpr int NG = (NB + 15) / 16;       // groups of 16 blocks (MFMA columns)
    static constexpr int UH = (NU + kSfThreads - 1) / kSfThreads;    // halo loads per thread
    // thread mappings that keep a thread's factor rows fixed: the x pass gives
    // thread t the column x = t % TX (XA threads, rows strided by XR); the y
    // pass and the tile points give thread t < YA the column (x, y) =
    // (t % TX, t / TX % TY) and the planes t / YT + YR k
    static constexpr int XR = kSfThreads / TX, XA = XR * TX;
    static constexpr int YT = TX * TY, YR = kSfThreads / YT, YA = YR * YT;
    static constexpr int PTS = TZ / YR;      // tile points per thread (q = t + YA k)
    static_assert(TZ % YR == 0, "tile planes must divide among the thread planes");
    static_assert(NR <= NT, "r and delta live in the tM / tK area");
};

// LDS index of point k (0..26, x fastest) of block n of the tile, in the
// tile-point layout [z][y][x]
template <int P>
__device__ __forceinline__ int sf_block_point(int n, int k) {
    using G = Sf<P>;
    const int bx = n % G::NBX, by = (n / G::NBX) % G::NBY, bz = n / (G::NBX * G::NBY);
    const int lx = k % 3, ly = (k / 3) % 3, lz = k / 9;
    return ((3 * bz + lz) * G::TY + 3 * by + ly) * G::TX + 3 * bx + lx;
}

// The x and y passes of A x on a tile: expects the iterate halo in sm[0, NU)
// and the factor rows in sm[OFF_F, ..) (K then M per row; x rows, then y rows,
// then z rows); leaves a and b in sm[OFF_A, ..), each pass followed by a
// barrier.  The z pass (sf_z) is evaluated per tile point by the caller.
template <int P, class T>
__device__ __forceinline__ void sf_apply(T *sm) {
    using G = Sf<P>;
    constexpr int W1 = G::W1;
    const int t = threadIdx.x;
    const T *xs = sm;
    T *tM = sm + G::OFF_T, *tK = tM + G::NT;
    const T *fx = sm + G::OFF_F, *fy = fx + G::TX * 2 * W1;
    // x pass: tM, tK at (x, hy, hz) for the tile's x and the halo's y, z
    if (t < G::XA) {
        const int x = t % G::TX;
        T kr[W1], mr[W1];
#pragma unroll
        for (int o = 0; o < W1; ++o) {
            kr[o] = fx[x * 2 * W1 + o];
            mr[o] = fx[x * 2 * W1 + W1 + o];
        }
        for (int row = t / G::TX; row < G::HY * G::HZ; row += G::XR) {
            const T *xr = xs + row * G::HX + x;
            T am = T(0), ak = T(0);
#pragma unroll
            for (int o = 0; o < W1; ++o) {
                const T v = xr[o];
                am += mr[o] * v;
                ak += kr[o] * v;
            }
            tM[row * G::TX + x] = am;
            tK[row * G::TX + x] = ak;
        }
    }
    __syncthreads();
    // y pass: a = My tM, b = Ky tM + My tK at (x, y, hz)
    T *a = sm + G::OFF_A, *b = a + G::NA;
    if (t < G::YA) {
        const int x = t % G::TX, y = (t / G::TX) % G::TY;
        T kr[W1], mr[W1];
#pragma unroll
        for (int o = 0; o < W1; ++o) {
            kr[o] = fy[y * 2 * W1 + o];
            mr[o] = fy[y * 2 * W1 + W1 + o];
        }
        for (int hz = t / G::YT; hz < G::HZ; hz += G::YR) {
            const int base = (hz * G::HY + y) * G::TX + x;
            T va = T(0), vb = T(0);
#pragma unroll
            for (int o = 0; o < W1; ++o) {
                const T m = tM[base + o * G::TX], k = tK[base + o * G::TX];
                va += mr[o] * m;
                vb += kr[o] * m + mr[o] * k;
            }
            a[(hz * G::TY + y) * G::TX + x] = va;
            b[(hz * G::TY + y) * G::TX + x] = vb;
        }
    }
    __syncthreads();
}

// z pass for tile point q: A x = Kz a + Mz b
template <int P, class T>
__device__ __forceinline__ T sf_z(const T *sm, int q) {
    using G = Sf<P>;
    constexpr int W1 = G::W1;
    const T *a = sm + G::OFF_A, *b = a + G::NA;
    const T *fz = sm + G::OFF_F + (G::TX + G::TY) * 2 * W1;
    const int xy = q % (G::TX * G::TY), z = q / (G::TX * G::TY);
    const T *kr = fz + z * 2 * W1, *mr = kr + W1;
    T acc = T(0);
#pragma unroll
    for (int o = 0; o < W1; ++o) {
        const int i = (z + o) * G::TX * G::TY + xy;
        acc += kr[o] * a[i] + mr[o] * b[i];
    }
    return acc;
}

// stage the iterate halo (zeros outside the grid) and the factor rows
template <int P, class T>
__device__ __forceinline__ void sf_stage(T *sm, const T *__restrict__ x, const T *__restrict__ kron, int n1, int gx0,
                                         int gy0, int gz0) {
    using G = Sf<P>;
    constexpr int W1 = G::W1;
    T *f = sm + G::OFF_F;
    for (int i = threadIdx.x; i < G::NF; i += kSfThreads) {
        const int row = i / (2 * W1), c = i % (2 * W1);
        const int g = row < G::TX ? gx0 + row : (row < G::TX + G::TY ? gy0 + row - G::TX : gz0 + row - G::TX - G::TY);
        const bool in = g >= 0 && g < n1;
        // kron = K1 [n1][W1] then M1 [n1][W1]
        f[i] = in ? kron[(c < W1 ? int64_t(0) : int64_t(n1) * W1) + int64_t(g) * W1 + (c % W1)] : T(0);
    }
    // every halo load of a thread is issued before its first LDS store: one memory round trip
    stage_lds<G::UH, T>(sm, G::NU, [&](int h) -> T {
        const int hx = h % G::HX, hy = (h / G::HX) % G::HY, hz = h / (G::HX * G::HY);
        const int gx = gx0 + hx - P, gy = gy0 + hy - P, gz = gz0 + hz - P;
        const bool in = gx >= 0 && gx < n1 && gy >= 0 && gy < n1 && gz >= 0 && gz < n1;
        return in ? x[(int64_t(gz) * n1 + gy) * n1 + gx] : T(0);
    });
}

// tile point q (x fastest) of the tile with origin (gx0, gy0, gz0) inside the grid
template <int P>
__device__ __forceinline__ bool in_grid3(int gx0, int gy0, int gz0, int q, int n1) {
    using G = Sf<P>;
    const int gx = gx0 + q % G::TX, gy = gy0 + (q / G::TX) % G::TY, gz = gz0 + q / G::YT;
    return gx >= 0 && gx < n1 && gy >= 0 && gy < n1 && gz >= 0 && gz < n1;
}

// tile -> workgroup: tiles dealt to the XCDs in contiguous bands
__device__ __forceinline__ void sf_tile(int ntx, int nty, int ntz, int &tx, int &ty, int &tz) {
    int L, dummy;
    const int nb = ntx * nty * ntz;
    xcd_relabel(int(blockIdx.x), nb, nb, L, dummy);
    tx = L % ntx;
    ty = (L / ntx) % nty;
    tz = L / (ntx * nty);
}

// 16x16x4 MFMA: lane l supplies A[l%16][l/16] and B[l/16][l%16]; value v of
// its result is D[row(l, v)][l%16] (the FP32 and FP64 instructions order the
// rows differently; both checked on the device)
template <class T>
struct MfmaAcc;
template <>
struct MfmaAcc<float> {
    using V = sf_f4;
    static __device__ __forceinline__ V step(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane / 16) + v; }
};
template <>
struct MfmaAcc<double> {
    using V = sf_d4;
    static __device__ __forceinline__ V step(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return lane / 16 + 4 * v; }
};

// One colour (cx, cy, cz) of the Schwarz sweep, colour period 3, 3x3x3 blocks,
// kappa = 1.  x_zero: the colour-start iterate is zero (no halo, r = rhs);
// r64 (with x_zero): the right-hand side is r64 / sigma, also stored to rhs_out.
template <int P, class T>
__global__ void __launch_bounds__(kSfThreads, 4) k_colour3d_sf(
    const T *__restrict__ kron, int n1, const T *__restrict__ inv, int clsL, int ncls1, const T *__restrict__ x_src,
    T *__restrict__ x_dst, const T *__restrict__ rhs, int x_zero, int ox, int oy, int oz, int ntx, int nty, int ntz,
    const int *__restrict__ skip, const double *__restrict__ r64, const double *__restrict__ scal,
    T *__restrict__ rhs_out) {
    using G = Sf<P>;
    extern __shared__ unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    const int stop = skip ? *skip : 0;   // tested before the first store
    int tbx, tby, tbz;
    sf_tile(ntx, nty, ntz, tbx, tby, tbz);
    const int gx0 = ox + tbx * G::TX, gy0 = oy + tby * G::TY, gz0 = oz + tbz * G::TZ;
    const int t = threadIdx.x, lane = t % 64, wave = t / 64;
    // this thread's tile points q = t + YA k: right-hand side, iterate and the
    // block each belongs to, issued with the halo
    T rv[G::PTS], xv[G::PTS];
    // per point: -2 outside the grid or in no block of the colour, -1 interior
    // block (MFMA), else the offset of its inverse row (boundary block)
    int64_t rowoff[G::PTS];
#pragma unroll
    for (int k = 0; k < G::PTS; ++k) {
        const int q = t + k * G::YA;
        const int x = q % G::TX, y = (q / G::TX) % G::TY, z = q / G::YT;
        const int gx = gx0 + x, gy = gy0 + y, gz = gz0 + z;
        const bool in = t < G::YA && gx >= 0 && gx < n1 && gy >= 0 && gy < n1 && gz >= 0 && gz < n1;
        const int64_t gi = in ? (int64_t(gz) * n1 + gy) * n1 + gx : 0;
        rv[k] = T(0);
        xv[k] = T(0);
        rowoff[k] = -2;
        if (in) {
            if (r64) rv[k] = T(r64[gi] * scal[kScalInvSigma]);
            else rv[k] = rhs[gi];
            if (!x_zero) xv[k] = x_src[gi];
            const int ccx = gx0 + 3 * (x / 3) + 1, ccy = gy0 + 3 * (y / 3) + 1, ccz = gz0 + 3 * (z / 3) + 1;
            if (ccx >= 0 && ccx < n1 && ccy >= 0 && ccy < n1 && ccz >= 0 && ccz < n1) {
                const int cx = clsL >= 0 ? block_class(ccx, n1, clsL) : ccx;
                const int cy = clsL >= 0 ? block_class(ccy, n1, clsL) : ccy;
                const int cz = clsL >= 0 ? block_class(ccz, n1, clsL) : ccz;
                if (clsL >= 0 && cx == clsL && cy == clsL && cz == clsL) {
                    rowoff[k] = -1;
                } else {
                    const int64_t slot = cx + int64_t(ncls1) * cy + int64_t(ncls1) * ncls1 * cz;
                    const int loc = (x % 3) + 3 * (y % 3) + 9 * (z % 3);
                    rowoff[k] = (slot * 27 + loc) * 27;
                }
            }
        }
    }
    // the interior inverse rows this wave multiplies (A operand of its MFMA jobs)
    const bool mfma = clsL >= 0;
    const int mt = wave % 2;    // M tile (block points 0..15 or 16..31) of this wave's jobs
    T ainv[7];
    if (mfma && wave / 2 < G::NG) {
        const int64_t slot = int64_t(clsL) * (1 + ncls1 + int64_t(ncls1) * ncls1);
        const int i = mt * 16 + lane % 16;
#pragma unroll
        for (int s = 0; s < 7; ++s) {
            const int k = 4 * s + lane / 16;
            ainv[s] = (i < 27 && k < 27) ? inv[(slot * 27 + i) * 27 + k] : T(0);
        }
    }
    T *r = sm + G::OFF_R, *delta = sm + G::OFF_D;
    if (!x_zero) {
        sf_stage<P, T>(sm, x_src, kron, n1, gx0, gy0, gz0);
        __syncthreads();
        sf_apply<P, T>(sm);
        // z pass: r = rhs - A x (0 outside the grid); tM / tK are dead, r takes their place
#pragma unroll
        for (int k = 0; k < G::PTS; ++k)
            if (t < G::YA)
                rv[k] = in_grid3<P>(gx0, gy0, gz0, t + k * G::YA, n1) ? rv[k] - sf_z<P, T>(sm, t + k * G::YA) : T(0);
    }
#pragma unroll
    for (int k = 0; k < G::PTS; ++k)
        if (t < G::YA) r[t + k * G::YA] = rv[k];
    __syncthreads();
    // interior blocks: delta = Inv R on the matrix cores, jobs (group of 16
    // blocks, M tile) dealt to the waves
    if (mfma) {
        using V = typename MfmaAcc<T>::V;
        for (int g = wave / 2; g < G::NG; g += kSfWaves / 2) {
            const int n = g * 16 + lane % 16;
            V acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int s = 0; s < 7; ++s) {
                const int k = 4 * s + lane / 16;
                const T bv = (n < G::NB && k < 27) ? r[sf_block_point<P>(n, k)] : T(0);
                acc = MfmaAcc<T>::step(ainv[s], bv, acc);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = mt * 16 + MfmaAcc<T>::row(lane, v);
                if (i < 27 && n < G::NB) delta[sf_block_point<P>(n, i)] = acc[v];
            }
        }
    }
    __syncthreads();
    if (stop) return;
    // update: x_dst = x + delta; blocks outside the interior class on the vector units
#pragma unroll
    for (int k = 0; k < G::PTS; ++k) {
        const int q = t + k * G::YA;
        if (t >= G::YA || !in_grid3<P>(gx0, gy0, gz0, q, n1)) continue;
        const int x = q % G::TX, y = (q / G::TX) % G::TY, z = q / G::YT;
        const int64_t gi = (int64_t(gz0 + z) * n1 + gy0 + y) * n1 + gx0 + x;
        if (r64) rhs_out[gi] = rv[k];
        T d = T(0);
        if (rowoff[k] == -1) {
            d = delta[q];
        } else if (rowoff[k] >= 0) {
            const int nblk = ((z / 3) * G::NBY + y / 3) * G::NBX + x / 3;
            // (loading these rows ahead into registers measured slower: occupancy)
#pragma unroll
            for (int l = 0; l < 27; ++l) d += inv[rowoff[k] + l] * r[sf_block_point<P>(nblk, l)];
        }
        x_dst[gi] = xv[k] + d;
    }
}

// Residual r = b - A x (kappa = 1) on tiles of Sf<P> points; NORM: per-
// workgroup sums of r^2 into partial[workgroup] (combined in a fixed order).
template <int P, class T, bool NORM>
__global__ void __launch_bounds__(kSfThreads) k_residual3d_sf(const T *__restrict__ kron, int n1,
                                                              const T *__restrict__ x, const T *__restrict__ b,
                                                              T *__restrict__ r, double *__restrict__ partial,
                                                              int ntx, int nty, int ntz,
                                                              const int *__restrict__ skip) {
    using G = Sf<P>;
    extern __shared__ unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    const int stop = skip ? *skip : 0;
    int tbx, tby, tbz;
    sf_tile(ntx, nty, ntz, tbx, tby, tbz);
    const int gx0 = tbx * G::TX, gy0 = tby * G::TY, gz0 = tbz * G::TZ;
    const int t = threadIdx.x;
    T bv[G::PTS];
#pragma unroll
    for (int k = 0; k < G::PTS; ++k) {
        const int q = t + k * G::YA;
        const int gx = gx0 + q % G::TX, gy = gy0 + (q / G::TX) % G::TY, gz = gz0 + q / G::YT;
        const bool in = t < G::YA && gx < n1 && gy < n1 && gz < n1;
        bv[k] = in ? b[(int64_t(gz) * n1 + gy) * n1 + gx] : T(0);
    }
    sf_stage<P, T>(sm, x, kron, n1, gx0, gy0, gz0);
    __syncthreads();
    sf_apply<P, T>(sm);
    double rr = 0.0;
#pragma unroll
    for (int k = 0; k < G::PTS; ++k) {
        const int q = t + k * G::YA;
        const int gx = gx0 + q % G::TX, gy = gy0 + (q / G::TX) % G::TY, gz = gz0 + q / G::YT;
        if (t < G::YA && gx < n1 && gy < n1 && gz < n1) {
            const T res = bv[k] - sf_z<P, T>(sm, q);
            if (!stop) r[(int64_t(gz) * n1 + gy) * n1 + gx] = res;
            rr += double(res) * double(res);
        }
    }
    if (stop) return;
    if constexpr (NORM) {
        __shared__ double red[kSfWaves];
        for (int off = 32; off > 0; off >>= 1) rr += __shfl_down(rr, off, 64);
        if ((threadIdx.x % 64) == 0) red[threadIdx.x / 64] = rr;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int k = 0; k < kSfWaves; ++k) s += red[k];
            partial[blockIdx.x] = s;
        }
    }
}

template <class T>
const T *kron_of(const Problem &P) {
    return std::is_same<T, double>::value ? reinterpret_cast<const T *>(P.kron64.ptr)
                                          : reinterpret_cast<const T *>(P.kron32.ptr);
}

// more than 64 KiB of dynamic LDS (FP64 tiles) must be allowed per kernel
template <class K>
void allow_lds(K kern, size_t bytes, bool &done) {
    if (done || bytes <= 65536) return;
    IGA2L_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  int(bytes)));
    done = true;
}

template <int P, class T>
void colour3d_launch(const Problem &Pb, int cx, int cy, int cz, const T *x_src, T *x_dst, const T *rhs, bool x_zero,
                     const double *r64, T *rhs_out, hipStream_t s) {
    using G = Sf<P>;
    static bool lds_done = false;
    allow_lds(k_colour3d_sf<P, T>, size_t(G::LDS) * sizeof(T), lds_done);
    const int n1 = Pb.fine.n1;
    // tile origins aligned with the colour's blocks, at or before index 0
    int ox = cx - 1, oy = cy - 1, oz = cz - 1;
    if (ox > 0) ox -= 3;
    if (oy > 0) oy -= 3;
    if (oz > 0) oz -= 3;
    const int ntx = (n1 - ox + G::TX - 1) / G::TX, nty = (n1 - oy + G::TY - 1) / G::TY,
              ntz = (n1 - oz + G::TZ - 1) / G::TZ;
    const T *inv = std::is_same<T, double>::value ? reinterpret_cast<const T *>(Pb.Inv64.ptr)
                                                  : reinterpret_cast<const T *>(Pb.Inv32.ptr);
    hipLaunchKernelGGL((k_colour3d_sf<P, T>), dim3(ntx * nty * ntz), dim3(kSfThreads), size_t(G::LDS) * sizeof(T), s,
                       kron_of<T>(Pb), n1, inv, class_split(Pb), Pb.ncls1, x_src, x_dst, rhs, x_zero ? 1 : 0, ox, oy,
                       oz, ntx, nty, ntz, Pb.skip, r64, Pb.scal.as<double>(), rhs_out);
}

template <int P, class T, bool NORM>
void residual3d_launch(const Problem &Pb, const T *x, const T *b, T *r, double *partial, hipStream_t s) {
    using G = Sf<P>;
    static bool lds_done = false;
    allow_lds(k_residual3d_sf<P, T, NORM>, size_t(G::LDS) * sizeof(T), lds_done);
    const int n1 = Pb.fine.n1;
    const int ntx = (n1 + G::TX - 1) / G::TX, nty = (n1 + G::TY - 1) / G::TY, ntz = (n1 + G::TZ - 1) / G::TZ;
    hipLaunchKernelGGL((k_residual3d_sf<P, T, NORM>), dim3(ntx * nty * ntz), dim3(kSfThreads),
                       size_t(G::LDS) * sizeof(T), s, kron_of<T>(Pb), n1, x, b, r, partial, ntx, nty, ntz, Pb.skip);
}

}  // namespace

bool colour3d_sf_ok(const Problem &P, int S) {
    return P.dim == 3 && P.bw == 3 && S == 3 && P.kron64.ptr != nullptr && P.p >= 1 && P.p <= 4;
}

bool residual3d_sf_ok(const Problem &P) { return P.dim == 3 && P.kron64.ptr != nullptr && P.p >= 1 && P.p <= 4; }

int64_t residual3d_sf_workgroups(const Problem &P) {
    const int64_t n1 = P.fine.n1;
    // the tile shape does not depend on p
    return ((n1 + Sf<1>::TX - 1) / Sf<1>::TX) * ((n1 + Sf<1>::TY - 1) / Sf<1>::TY) * ((n1 + Sf<1>::TZ - 1) / Sf<1>::TZ);
}

template <class T>
void launch_colour3d_sf(const Problem &Pb, int cx, int cy, int cz, const T *x_src, T *x_dst, const T *rhs,
                        bool x_zero, const double *r64, T *rhs_out, hipStream_t s) {
    switch (Pb.p) {
        case 1: colour3d_launch<1, T>(Pb, cx, cy, cz, x_src, x_dst, rhs, x_zero, r64, rhs_out, s); break;
        case 2: colour3d_launch<2, T>(Pb, cx, cy, cz, x_src, x_dst, rhs, x_zero, r64, rhs_out, s); break;
        case 3: colour3d_launch<3, T>(Pb, cx, cy, cz, x_src, x_dst, rhs, x_zero, r64, rhs_out, s); break;
        case 4: colour3d_launch<4, T>(Pb, cx, cy, cz, x_src, x_dst, rhs, x_zero, r64, rhs_out, s); break;
        default: throw Error{IGA2L_EUNSUPPORTED, "3-D degree out of range"};
    }
}
template void launch_colour3d_sf<double>(const Problem &, int, int, int, const double *, double *, const double *,
                                         bool, const double *, double *, hipStream_t);
template void launch_colour3d_sf<float>(const Problem &, int, int, int, const float *, float *, const float *, bool,
                                        const double *, float *, hipStream_t);

template <class T, bool NORM>
void launch_residual3d_sf(const Problem &Pb, const T *x, const T *b, T *r, double *partial, hipStream_t s) {
    switch (Pb.p) {
        case 1: residual3d_launch<1, T, NORM>(Pb, x, b, r, partial, s); break;
        case 2: residual3d_launch<2, T, NORM>(Pb, x, b, r, partial, s); break;
        case 3: residual3d_launch<3, T, NORM>(Pb, x, b, r, partial, s); break;
        case 4: residual3d_launch<4, T, NORM>(Pb, x, b, r, partial, s); break;
        default: throw Error{IGA2L_EUNSUPPORTED, "3-D degree out of range"};
    }
}
template void launch_residual3d_sf<double, true>(const Problem &, const double *, const double *, double *, double *,
                                                 hipStream_t);
template void launch_residual3d_sf<double, false>(const Problem &, const double *, const double *, double *,
                                                  double *, hipStream_t);
template void launch_residual3d_sf<float, false>(const Problem &, const float *, const float *, float *, double *,
                                                 hipStream_t);
template void launch_residual3d_sf<float, true>(const Problem &, const float *, const float *, float *, double *,
                                                hipStream_t);

}  // namespace iga2l
