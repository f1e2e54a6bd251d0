// kernels_coarse.hip -- transfer, coarse-level and auxiliary kernels of the
// two-level solver on gfx950: restriction by the lumped L2 projection and its
// adjoint prolongation (tensor products of the 1-D factor R1), the exact
// coarse solve for kappa = 1 by DST-I diagonalisation, precision conversions
// and the element-wise kappa-gradient of the adjoint.  The V-cycle lives in
// kernels_vcycle.hip.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace iga2l {

namespace {

inline unsigned nblocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

// ------------------------------------------------------------ transfers --
// d_c[I] = sum_a R1[Ix][ax] R1[Iy][ay] (R1[Iz][az]) d[I - plow + a],
// a in [0, p+plow]^D (coarse space of degree plow)
template <int D, class T>
__global__ void k_restrict(const T *__restrict__ R1, const T *__restrict__ R1y, int p, int plow, int n1f, int n1c,
                           const T *__restrict__ df, T *__restrict__ dc, const int *__restrict__ skip) {
    const int stop = skip ? *skip : 0;  // tested before the store (hides the load latency)
    const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nc = (D == 3) ? int64_t(n1c) * n1c * n1c : int64_t(n1c) * n1c;
    if (I >= nc) return;
    const int Ix = int(I % n1c), Iy = int((I / n1c) % n1c), Iz = (D == 3) ? int(I / (int64_t(n1c) * n1c)) : 0;
    const int w = p + plow + 1;
    T acc = T(0);
    for (int az = 0; az < ((D == 3) ? w : 1); ++az) {
        const int jz = (D == 3) ? Iz - plow + az : 0;
        if (D == 3 && (jz < 0 || jz >= n1f)) continue;
        const T rz = (D == 3) ? R1y[Iz * w + az] : T(1);
        for (int ay = 0; ay < w; ++ay) {
            const int jy = Iy - plow + ay;
            if (jy < 0 || jy >= n1f) continue;
            const T ry = R1y[Iy * w + ay] * rz;
            T line = T(0);
            for (int ax = 0; ax < w; ++ax) {
                const int jx = Ix - plow + ax;
                if (jx < 0 || jx >= n1f) continue;
                line += R1[Ix * w + ax] * df[(int64_t(jz) * n1f + jy) * n1f + jx];
            }
            acc += ry * line;
        }
    }
    if (stop) return;
    dc[I] = acc;
}

// (P e_c)[i] = sum over coarse I with i - I + plow in [0,p+plow] per direction
// of R1[Ix][ix-Ix+plow] R1[Iy][iy-Iy+plow] (..) e_c[I]: the exact transpose of
// k_restrict.
template <int D, class T>
__device__ __forceinline__ T prolong_value(const T *__restrict__ R1, const T *__restrict__ R1y, int p, int plow,
                                           int n1f, int n1c, const T *__restrict__ ec, int ix, int iy, int iz) {
    const int w = p + plow + 1;
    T acc = T(0);
    for (int Iz = ((D == 3) ? iz - p : 0); Iz <= ((D == 3) ? iz + plow : 0); ++Iz) {
        if (D == 3 && (Iz < 0 || Iz >= n1c)) continue;
        const T rz = (D == 3) ? R1y[Iz * w + (iz - Iz + plow)] : T(1);
        for (int Iy = iy - p; Iy <= iy + plow; ++Iy) {
            if (Iy < 0 || Iy >= n1c) continue;
            const T ry = R1y[Iy * w + (iy - Iy + plow)] * rz;
            T line = T(0);
            for (int Ix = ix - p; Ix <= ix + plow; ++Ix) {
                if (Ix < 0 || Ix >= n1c) continue;
                line += R1[Ix * w + (ix - Ix + plow)] * ec[(int64_t(Iz) * n1c + Iy) * n1c + Ix];
            }
            acc += ry * line;
        }
    }
    return acc;
}

template <int D, class T>
__global__ void k_prolong_add(const T *__restrict__ R1, const T *__restrict__ R1y, int p, int plow, int n1f, int n1c,
                              const T *__restrict__ ec, T *__restrict__ uf, const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nf = (D == 3) ? int64_t(n1f) * n1f * n1f : int64_t(n1f) * n1f;
    if (i >= nf) return;
    const int ix = int(i % n1f), iy = int((i / n1f) % n1f), iz = (D == 3) ? int(i / (int64_t(n1f) * n1f)) : 0;
    uf[i] += prolong_value<D, T>(R1, R1y, p, plow, n1f, n1c, ec, ix, iy, iz);
}

// u64 += sigma * (e + P e_c): end of a correction cycle
template <int D, class T>
__global__ void k_prolong_update(const T *__restrict__ R1, const T *__restrict__ R1y, int p, int plow, int n1f,
                                 int n1c, const T *__restrict__ ec, const T *__restrict__ e, double *__restrict__ u,
                                 const double *__restrict__ scal, int scaled, const int *__restrict__ skip) {
    const int stop = skip ? *skip : 0;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nf = (D == 3) ? int64_t(n1f) * n1f * n1f : int64_t(n1f) * n1f;
    if (i >= nf) return;
    const int ix = int(i % n1f), iy = int((i / n1f) % n1f), iz = (D == 3) ? int(i / (int64_t(n1f) * n1f)) : 0;
    const T corr = e[i] + prolong_value<D, T>(R1, R1y, p, plow, n1f, n1c, ec, ix, iy, iz);
    if (stop) return;
    u[i] += scaled ? scal[kScalSigma] * double(corr) : double(corr);
}

// ----------------------------------------------------------------- DST --
// out[.., k, ..] = sum_i S[k][i] in[.., i, ..] along one axis (S row-major);
// with mu != nullptr the result is divided by mu (diagonal solve).
__global__ void k_dst_axis(const double *__restrict__ S, int n1, int dim, int axis, const double *__restrict__ in,
                           double *__restrict__ out, const double *__restrict__ mu, const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int64_t n = (dim == 3) ? int64_t(n1) * n1 * n1 : int64_t(n1) * n1;
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    int64_t stride = 1;
    for (int k = 0; k < axis; ++k) stride *= n1;
    const int k = int((idx / stride) % n1);
    const int64_t base = idx - int64_t(k) * stride;
    const double *Srow = S + int64_t(k) * n1;
    double acc = 0.0;
    for (int i = 0; i < n1; ++i) acc += Srow[i] * in[base + int64_t(i) * stride];
    out[idx] = mu ? acc / mu[idx] : acc;
}

template <class T>
__global__ void k_fill(T *__restrict__ x, int64_t n, const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) x[i] = T(0);
}

template <class A, class B>
__global__ void k_convert(const A *__restrict__ a, B *__restrict__ b, int64_t n, const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) b[i] = B(a[i]);
}

// ------------------------------------------------------------ gradient --
// g_e = - lambda_e^T K_e u_e with the unit-coefficient element stiffness
// K_e = sum_c (x)_k (k == c ? K^{1D}_{e_k} : M^{1D}_{e_k}); this is
// -integral_e grad(lambda_h) . grad(u_h).
template <int D>
__global__ void k_grad_kappa(const double *__restrict__ KM, int p, int m, int n1, const double *__restrict__ u,
                             const double *__restrict__ lam, double *__restrict__ g) {
    const int64_t ne = (D == 3) ? int64_t(m) * m * m : int64_t(m) * m;
    const int64_t el = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (el >= ne) return;
    const int ex = int(el % m), ey = int((el / m) % m), ez = (D == 3) ? int(el / (int64_t(m) * m)) : 0;
    const int nl = p + 1, nl2 = nl * nl;
    const double *Kx = KM + (int64_t(ex) * 2 + 0) * nl2, *Mx = KM + (int64_t(ex) * 2 + 1) * nl2;
    const double *Ky = KM + (int64_t(ey) * 2 + 0) * nl2, *My = KM + (int64_t(ey) * 2 + 1) * nl2;
    const double *Kz = KM + (int64_t(ez) * 2 + 0) * nl2, *Mz = KM + (int64_t(ez) * 2 + 1) * nl2;
    double acc = 0.0;
    for (int az = 0; az < ((D == 3) ? nl : 1); ++az)
        for (int ay = 0; ay < nl; ++ay)
            for (int ax = 0; ax < nl; ++ax) {
                const int ix = ex + ax - 1, iy = ey + ay - 1, iz = (D == 3) ? ez + az - 1 : 0;
                if (ix < 0 || ix >= n1 || iy < 0 || iy >= n1 || (D == 3 && (iz < 0 || iz >= n1))) continue;
                const double la = lam[(int64_t(iz) * n1 + iy) * n1 + ix];
                double row = 0.0;
                for (int bz = 0; bz < ((D == 3) ? nl : 1); ++bz)
                    for (int by = 0; by < nl; ++by)
                        for (int bx = 0; bx < nl; ++bx) {
                            const int jx = ex + bx - 1, jy = ey + by - 1, jz = (D == 3) ? ez + bz - 1 : 0;
                            if (jx < 0 || jx >= n1 || jy < 0 || jy >= n1 || (D == 3 && (jz < 0 || jz >= n1))) continue;
                            double kab;
                            if (D == 2) {
                                kab = Kx[ax * nl + bx] * My[ay * nl + by] + Mx[ax * nl + bx] * Ky[ay * nl + by];
                            } else {
                                kab = Kx[ax * nl + bx] * My[ay * nl + by] * Mz[az * nl + bz] +
                                      Mx[ax * nl + bx] * Ky[ay * nl + by] * Mz[az * nl + bz] +
                                      Mx[ax * nl + bx] * My[ay * nl + by] * Kz[az * nl + bz];
                            }
                            row += kab * u[(int64_t(jz) * n1 + jy) * n1 + jx];
                        }
                acc += la * row;
            }
    g[el] = -acc;
}

// --------------------------------------------------------------- assembly --
// Upper diagonals of A = sum_e kappa_e A_e in the symmetric padded-diagonal
// form, one thread per (row, offset).  In each direction the elements shared
// by the supports of B-splines i and j = i + o are e = max(i,j)+1-p .. min(i,j)+1
// (0-based interior indices, element e covers [e/m, (e+1)/m]); the local
// indices are i+1-e and j+1-e, and the element matrix is the tensor product
// of the 1-D stiffness and mass matrices K1_e, M1_e (sum over the direction
// that carries the derivative).  Elements are summed in increasing index
// order.  val must be zero on entry (entries outside the grid stay zero).
template <int D>
__global__ void k_assemble_dia(const double *__restrict__ KM, const double *__restrict__ kappa, int p, int m, int n1,
                               int64_t npad, int pitch1, int pitch2, int c0, double *__restrict__ val) {
    const int64_t n = (D == 3) ? int64_t(n1) * n1 * n1 : int64_t(n1) * n1;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int wu = int(blockIdx.y);            // upper offset index (0 = centre)
    const int w1 = 2 * p + 1, w = c0 + wu;
    const int o[3] = {w % w1 - p, (w / w1) % w1 - p, (D == 3) ? w / (w1 * w1) - p : 0};
    const int ic[3] = {int(i % n1), int((i / n1) % n1), (D == 3) ? int(i / (int64_t(n1) * n1)) : 0};
    int elo[3] = {0, 0, 0}, ehi[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) {
        const int j = ic[k] + o[k];
        if (j < 0 || j >= n1) return;
        elo[k] = max(max(ic[k], j) + 1 - p, 0);
        ehi[k] = min(min(ic[k], j) + 1, m - 1);
    }
    const int nl = p + 1, nl2 = nl * nl;
    double acc = 0.0;
    for (int ez = elo[2]; ez <= ehi[2]; ++ez)
        for (int ey = elo[1]; ey <= ehi[1]; ++ey)
            for (int ex = elo[0]; ex <= ehi[0]; ++ex) {
                const int e[3] = {ex, ey, ez};
                double term = 0.0;
                for (int c = 0; c < D; ++c) {
                    double prod = 1.0;
                    for (int k = 0; k < D; ++k) {
                        const int a = ic[k] + 1 - e[k], b = ic[k] + o[k] + 1 - e[k];
                        prod *= KM[(int64_t(e[k]) * 2 + (k == c ? 0 : 1)) * nl2 + a * nl + b];
                    }
                    term += prod;
                }
                const int64_t el = (D == 3) ? (int64_t(ez) * m + ey) * m + ex : int64_t(ey) * m + ex;
                acc += kappa[el] * term;
            }
    const int64_t padi = int64_t(ic[0] + p) + int64_t(ic[1] + p) * pitch1 + ((D == 3) ? int64_t(ic[2] + p) * pitch2 : 0);
    val[int64_t(wu) * npad + padi] = acc;
}

// Full 3^d stencil of the degree-1 operator on the same knots, S[w][i]
// (w = offset index, x fastest), from the 1-D degree-1 element matrices KM1
// ([m][2][4], K then M) and kappa; same element rule as k_assemble_dia.
template <int D>
__global__ void k_assemble_q1(const double *__restrict__ KM1, const double *__restrict__ kappa, int m,
                              double *__restrict__ S) {
    const int n1 = m - 1;
    const int64_t n = (D == 3) ? int64_t(n1) * n1 * n1 : int64_t(n1) * n1;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int w = int(blockIdx.y);
    const int o[3] = {w % 3 - 1, (w / 3) % 3 - 1, (D == 3) ? w / 9 - 1 : 0};
    const int ic[3] = {int(i % n1), int((i / n1) % n1), (D == 3) ? int(i / (int64_t(n1) * n1)) : 0};
    int elo[3] = {0, 0, 0}, ehi[3] = {0, 0, 0};
    bool in = true;
    for (int k = 0; k < D; ++k) {
        const int j = ic[k] + o[k];
        if (j < 0 || j >= n1) in = false;
        elo[k] = max(ic[k], j);
        ehi[k] = min(min(ic[k], j) + 1, m - 1);
    }
    double acc = 0.0;
    if (in)
        for (int ez = elo[2]; ez <= ehi[2]; ++ez)
            for (int ey = elo[1]; ey <= ehi[1]; ++ey)
                for (int ex = elo[0]; ex <= ehi[0]; ++ex) {
                    const int e[3] = {ex, ey, ez};
                    double term = 0.0;
                    for (int c = 0; c < D; ++c) {
                        double prod = 1.0;
                        for (int k = 0; k < D; ++k) {
                            const int a = ic[k] + 1 - e[k], b = ic[k] + o[k] + 1 - e[k];
                            prod *= KM1[(int64_t(e[k]) * 2 + (k == c ? 0 : 1)) * 4 + a * 2 + b];
                        }
                        term += prod;
                    }
                    const int64_t el = (D == 3) ? (int64_t(ez) * m + ey) * m + ex : int64_t(ey) * m + ex;
                    acc += kappa[el] * term;
                }
    S[int64_t(w) * n + i] = acc;
}

// Galerkin coarse stencil Sc = P^T Sf P for linear interpolation from the
// odd-indexed fine nodes: coarse node J has the fine children 2J, 2J+1, 2J+2
// (weights 1/2, 1, 1/2 per direction, inside the fine grid).  One thread per
// (coarse row I, coarse offset W).
template <int D>
__global__ void k_galerkin(const double *__restrict__ Sf, int nf1, double *__restrict__ Sc, int nc1) {
    const int64_t nc = (D == 3) ? int64_t(nc1) * nc1 * nc1 : int64_t(nc1) * nc1;
    const int64_t nf = (D == 3) ? int64_t(nf1) * nf1 * nf1 : int64_t(nf1) * nf1;
    const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    const int W = int(blockIdx.y);
    const int Ic[3] = {int(I % nc1), int((I / nc1) % nc1), (D == 3) ? int(I / (int64_t(nc1) * nc1)) : 0};
    const int O[3] = {W % 3 - 1, (W / 3) % 3 - 1, (D == 3) ? W / 9 - 1 : 0};
    int Jc[3] = {0, 0, 0};
    bool in = true;
    for (int k = 0; k < D; ++k) {
        Jc[k] = Ic[k] + O[k];
        if (Jc[k] < 0 || Jc[k] >= nc1) in = false;
    }
    double acc = 0.0;
    if (in) {
        const double cw[3] = {0.5, 1.0, 0.5};
        for (int iz = 0; iz < ((D == 3) ? 3 : 1); ++iz)
            for (int iy = 0; iy < 3; ++iy)
                for (int ix = 0; ix < 3; ++ix) {
                    const int fi[3] = {2 * Ic[0] + ix, 2 * Ic[1] + iy, (D == 3) ? 2 * Ic[2] + iz : 0};
                    if (fi[0] >= nf1 || fi[1] >= nf1 || (D == 3 && fi[2] >= nf1)) continue;
                    const double wi = cw[ix] * cw[iy] * ((D == 3) ? cw[iz] : 1.0);
                    const int64_t fidx = (D == 3) ? (int64_t(fi[2]) * nf1 + fi[1]) * nf1 + fi[0]
                                                  : int64_t(fi[1]) * nf1 + fi[0];
                    for (int jz = 0; jz < ((D == 3) ? 3 : 1); ++jz)
                        for (int jy = 0; jy < 3; ++jy)
                            for (int jx = 0; jx < 3; ++jx) {
                                const int fj[3] = {2 * Jc[0] + jx, 2 * Jc[1] + jy, (D == 3) ? 2 * Jc[2] + jz : 0};
                                bool ok = true;
                                int wf = 0, mul = 1;
                                for (int k = 0; k < D; ++k) {
                                    const int dk = fj[k] - fi[k];
                                    if (fj[k] >= nf1 || dk < -1 || dk > 1) ok = false;
                                    wf += (dk + 1) * mul;
                                    mul *= 3;
                                }
                                if (!ok) continue;
                                const double wj = cw[jx] * cw[jy] * ((D == 3) ? cw[jz] : 1.0);
                                acc += wi * Sf[int64_t(wf) * nf + fidx] * wj;
                            }
                }
    }
    Sc[int64_t(W) * nc + I] = acc;
}

// the 1-D transfer factor: D1^{-1} Mmix1 (lumped), or Mmix1 when the exact
// transfers apply M_1^{-1} separately
// the factor of the y (and z) axis: the annulus's radial one, else R1
template <class T>
const T *R1y_of(const Problem &P);

template <class T>
const T *R1_of(const Problem &P) {
    if (P.transfer_exact)
        return std::is_same<T, double>::value ? reinterpret_cast<const T *>(P.Mx64.ptr)
                                              : reinterpret_cast<const T *>(P.Mx32.ptr);
    return std::is_same<T, double>::value ? reinterpret_cast<const T *>(P.R1d64.ptr)
                                          : reinterpret_cast<const T *>(P.R1d32.ptr);
}

template <class T>
const T *R1y_of(const Problem &P) {
    if (P.geometry != kGeomAnnulus) return R1_of<T>(P);
    return std::is_same<T, double>::value ? reinterpret_cast<const T *>(P.R1yd64.ptr)
                                          : reinterpret_cast<const T *>(P.R1yd32.ptr);
}

}  // namespace

// ------------------------------------------------------------ launchers --
// 2-D with the degree-1 coarse space: the tiled sum-factorised kernels of
// kernels_2d.hip; otherwise one thread per output point
template <class T>
void launch_restrict(const Problem &P, const T *df, T *dc, hipStream_t s) {
    if (P.dim == 2 && P.plow == 1 && P.geometry == kGeomSquare) {
        launch_restrict2d<T>(P, df, dc, s);
        return;
    }
    const int64_t nc = P.coarse.n;
    auto kern = P.dim == 2 ? k_restrict<2, T> : k_restrict<3, T>;
    hipLaunchKernelGGL(kern, dim3(nblocks(nc, 256)), dim3(256), 0, s, R1_of<T>(P), R1y_of<T>(P), P.p, P.plow,
                       P.fine.n1, P.coarse.n1, df, dc, P.skip);
}
template void launch_restrict<double>(const Problem &, const double *, double *, hipStream_t);
template void launch_restrict<float>(const Problem &, const float *, float *, hipStream_t);

template <class T>
void launch_prolong_add(const Problem &P, const T *ec, T *uf, hipStream_t s) {
    if (P.dim == 2 && P.plow == 1 && P.geometry == kGeomSquare) {
        launch_prolong2d<T>(P, ec, uf, nullptr, nullptr, false, s);
        return;
    }
    const int64_t nf = P.fine.n;
    auto kern = P.dim == 2 ? k_prolong_add<2, T> : k_prolong_add<3, T>;
    hipLaunchKernelGGL(kern, dim3(nblocks(nf, 256)), dim3(256), 0, s, R1_of<T>(P), R1y_of<T>(P), P.p, P.plow,
                       P.fine.n1, P.coarse.n1, ec, uf, P.skip);
}
template void launch_prolong_add<double>(const Problem &, const double *, double *, hipStream_t);
template void launch_prolong_add<float>(const Problem &, const float *, float *, hipStream_t);

template <class T>
void launch_prolong_update(const Problem &P, const T *ec, const T *e, double *u, bool scaled, hipStream_t s) {
    if (P.dim == 2 && P.plow == 1 && P.geometry == kGeomSquare) {
        launch_prolong2d<T>(P, ec, nullptr, e, u, scaled, s);
        return;
    }
    const int64_t nf = P.fine.n;
    auto kern = P.dim == 2 ? k_prolong_update<2, T> : k_prolong_update<3, T>;
    hipLaunchKernelGGL(kern, dim3(nblocks(nf, 256)), dim3(256), 0, s, R1_of<T>(P), R1y_of<T>(P), P.p, P.plow,
                       P.fine.n1, P.coarse.n1, ec, e, u, P.scal.as<double>(), scaled ? 1 : 0, P.skip);
}
template void launch_prolong_update<double>(const Problem &, const double *, const double *, double *, bool,
                                            hipStream_t);
template void launch_prolong_update<float>(const Problem &, const float *, const float *, double *, bool,
                                           hipStream_t);

// e = (S (x) .. (x) S) diag(mu)^{-1} (S (x) .. (x) S) d on a grid of n1^dim
// points (S symmetric orthogonal): forward transform along every axis,
// diagonal solve, inverse (= forward) transform.  t1: scratch of n doubles;
// d may equal t1 only if it is not e.
// Sb = nullptr: Sb = S (the DST-I is its own inverse); the fast
// diagonalisation of the degree-2 space passes V^T forward and V backward.
static void dst_apply(const double *S, const double *mu, int n1, int dim, const double *d, double *e, double *t1,
                      const int *skip, hipStream_t s, const double *Sb = nullptr, int64_t axis_stride = 0) {
    const int64_t n = (dim == 3) ? int64_t(n1) * n1 * n1 : int64_t(n1) * n1;
    const double *src = d;
    double *bufs[2] = {t1, e};
    int cur = 0;
    for (int ax = 0; ax < dim; ++ax) {
        hipLaunchKernelGGL(k_dst_axis, dim3(nblocks(n, 256)), dim3(256), 0, s, S + ax * axis_stride, n1, dim, ax, src,
                           bufs[cur], (ax == dim - 1) ? mu : nullptr, skip);
        src = bufs[cur];
        cur = 1 - cur;
    }
    for (int ax = 0; ax < dim; ++ax) {
        hipLaunchKernelGGL(k_dst_axis, dim3(nblocks(n, 256)), dim3(256), 0, s, (Sb ? Sb : S) + ax * axis_stride, n1,
                           dim, ax, src, bufs[cur], nullptr, skip);
        src = bufs[cur];
        cur = 1 - cur;
    }
    // 2*dim passes alternate t1, e, t1, e, ...: an even count, so the last one wrote e
}

// exact solve of level 1 (2h) of the hierarchy for aggressive coarsening
void dst_apply_2h(Problem &P, const double *d, double *e, double *t1, hipStream_t s) {
    dst_apply(P.dst2_S.as<double>(), P.dst2_mu.as<double>(), P.levels[1].g.n1, P.dim, d, e, t1, P.skip, s);
}

// e = Z d for a dense n x n matrix Z (row-major): one wavefront per row
__global__ void __launch_bounds__(256) k_dense_apply(const double *__restrict__ Z, int64_t n,
                                                     const double *__restrict__ d, double *__restrict__ e,
                                                     const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int64_t row = int64_t(blockIdx.x) * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (row >= n) return;  // whole wavefronts
    const double *z = Z + row * n;
    double acc = 0.0;
    for (int64_t j = lane; j < n; j += 64) acc += z[j] * d[j];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) e[row] = acc;
}

void launch_dst_solve(Problem &P, const double *d, double *e, hipStream_t s) {
    IGA2L_REQUIRE(P.direct_ready, IGA2L_EINVAL, "exact coarse solver not set up");
    if (P.plow == 1 && P.coarse_inv64.ptr) {
        // variable kappa: the inverse formed from the banded Cholesky factor
        const int64_t n = P.coarse.n;
        hipLaunchKernelGGL(k_dense_apply, dim3(unsigned((n + 3) / 4)), dim3(256), 0, s, P.coarse_inv64.as<double>(),
                           n, d, e, P.skip);
        return;
    }
    if (P.plow == 2)
        dst_apply(P.fdm_Vt.as<double>(), P.dst_mu.as<double>(), P.coarse.n1, P.dim, d, e, P.ctmp.as<double>(), P.skip,
                  s, P.fdm_V.as<double>(), P.fdm_axis_stride);
    else
        dst_apply(P.dst_S.as<double>(), P.dst_mu.as<double>(), P.coarse.n1, P.dim, d, e, P.ctmp.as<double>(), P.skip,
                  s);
}

// e = M_low^{-1} d: the DST-I of the degree-1 mass matrix, or the fast
// diagonalisation of the degree-2 space with unit eigenvalues (M2^{-1} = V V^T
// per direction)
static void mass_apply(Problem &P, const double *d, double *e, double *t1, hipStream_t s) {
    if (P.plow == 2)
        dst_apply(P.fdm_Vt.as<double>(), P.dstM_mu.as<double>(), P.coarse.n1, P.dim, d, e, t1, P.skip, s,
                  P.fdm_V.as<double>());
    else
        dst_apply(P.dstM_S.as<double>(), P.dstM_mu.as<double>(), P.coarse.n1, P.dim, d, e, t1, P.skip, s);
}

// x <- M_low^{-1} x (the coarse-space mass matrix, Dirichlet-reduced): FP64 through
// the DST-I; an FP32 x is widened, solved and narrowed
template <class T>
void launch_mass_solve(Problem &P, T *x, hipStream_t s) {
    IGA2L_REQUIRE(P.mass_ready, IGA2L_EINVAL, "exact transfers not set up (setup_blocks with lumped = 0)");
    const int64_t n = P.coarse.n;
    double *t1 = P.ctmp2.as<double>();
    if constexpr (std::is_same<T, double>::value) {
        // x -> e through t1: the input must not be the output buffer
        IGA2L_HIP(hipMemcpyAsync(P.ctmp.ptr, x, sizeof(double) * size_t(n), hipMemcpyDeviceToDevice, s));
        mass_apply(P, P.ctmp.as<double>(), x, t1, s);
    } else {
        IGA2L_REQUIRE(P.dc64.ptr, IGA2L_EINVAL, "FP32 data not set up");
        launch_convert(x, P.ctmp.ptr, n, false, s, P.skip);
        mass_apply(P, P.ctmp.as<double>(), P.dc64.as<double>(), t1, s);
        launch_convert(P.dc64.ptr, x, n, true, s, P.skip);
    }
}
template void launch_mass_solve<double>(Problem &, double *, hipStream_t);
template void launch_mass_solve<float>(Problem &, float *, hipStream_t);

void launch_convert(const void *src, void *dst, int64_t n, bool to_fp32, hipStream_t s, const int *skip) {
    if (to_fp32)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(nblocks(n, 256)), dim3(256), 0, s,
                           static_cast<const double *>(src), static_cast<float *>(dst), n, skip);
    else
        hipLaunchKernelGGL((k_convert<float, double>), dim3(nblocks(n, 256)), dim3(256), 0, s,
                           static_cast<const float *>(src), static_cast<double *>(dst), n, skip);
}

void launch_fill_zero(void *x, int64_t n_elems, bool fp32, hipStream_t s, const int *skip) {
    if (fp32)
        hipLaunchKernelGGL((k_fill<float>), dim3(nblocks(n_elems, 256)), dim3(256), 0, s, static_cast<float *>(x),
                           n_elems, skip);
    else
        hipLaunchKernelGGL((k_fill<double>), dim3(nblocks(n_elems, 256)), dim3(256), 0, s, static_cast<double *>(x),
                           n_elems, skip);
}

void launch_grad_kappa(const Problem &P, const double *u, const double *lam, double *g, hipStream_t s) {
    if (P.dim == 2)
        hipLaunchKernelGGL((k_grad_kappa<2>), dim3(nblocks(P.ne, 128)), dim3(128), 0, s, P.Ke_d.as<double>(), P.p, P.m,
                           P.fine.n1, u, lam, g);
    else
        hipLaunchKernelGGL((k_grad_kappa<3>), dim3(nblocks(P.ne, 128)), dim3(128), 0, s, P.Ke_d.as<double>(), P.p, P.m,
                           P.fine.n1, u, lam, g);
}

void launch_assemble_dia(Problem &P, hipStream_t s) {
    SymDia &A = P.A;
    const int c0 = (A.W - 1) / 2;
    IGA2L_HIP(hipMemsetAsync(A.v64.ptr, 0, size_t(A.Wh) * A.npad * sizeof(double), s));
    const dim3 grid(nblocks(P.fine.n, 256), unsigned(A.Wh));
    if (P.dim == 2)
        hipLaunchKernelGGL((k_assemble_dia<2>), grid, dim3(256), 0, s, P.Ke_d.as<double>(), P.kappa_d.as<double>(), P.p,
                           P.m, P.fine.n1, A.npad, A.pitch[1], A.pitch[2], c0, A.v64.as<double>());
    else
        hipLaunchKernelGGL((k_assemble_dia<3>), grid, dim3(256), 0, s, P.Ke_d.as<double>(), P.kappa_d.as<double>(), P.p,
                           P.m, P.fine.n1, A.npad, A.pitch[1], A.pitch[2], c0, A.v64.as<double>());
    IGA2L_HIP(hipGetLastError());
}

void launch_assemble_q1(int dim, const double *KM1, const double *kappa, int m, double *S, hipStream_t s) {
    const int n1 = m - 1;
    const int64_t n = (dim == 3) ? int64_t(n1) * n1 * n1 : int64_t(n1) * n1;
    const dim3 grid(nblocks(n, 256), dim == 3 ? 27 : 9);
    if (dim == 2) hipLaunchKernelGGL((k_assemble_q1<2>), grid, dim3(256), 0, s, KM1, kappa, m, S);
    else hipLaunchKernelGGL((k_assemble_q1<3>), grid, dim3(256), 0, s, KM1, kappa, m, S);
    IGA2L_HIP(hipGetLastError());
}

void launch_galerkin(int dim, const double *Sf, int nf1, double *Sc, int nc1, hipStream_t s) {
    const int64_t nc = (dim == 3) ? int64_t(nc1) * nc1 * nc1 : int64_t(nc1) * nc1;
    const dim3 grid(nblocks(nc, 256), dim == 3 ? 27 : 9);
    if (dim == 2) hipLaunchKernelGGL((k_galerkin<2>), grid, dim3(256), 0, s, Sf, nf1, Sc, nc1);
    else hipLaunchKernelGGL((k_galerkin<3>), grid, dim3(256), 0, s, Sf, nf1, Sc, nc1);
    IGA2L_HIP(hipGetLastError());
}

}  // namespace iga2l
