// kernels_coarse.hip -- transfer, coarse-level and auxiliary kernels of the
// two-level solver on gfx950: restriction by the lumped L2 projection and its
// adjoint prolongation (tensor products of the 1-D factor R1), the degree-1
// h-multigrid V-cycle (red-black Gauss-Seidel, linear interpolation, Galerkin
// operators), the exact coarse solve for kappa = 1 by DST-I diagonalisation,
// precision conversions and the element-wise kappa-gradient of the adjoint.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace iga2l {

namespace {

inline unsigned nblocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

// ------------------------------------------------------------ transfers --
// d_c[I] = sum_a R1[Ix][ax] R1[Iy][ay] (R1[Iz][az]) d[I - 1 + a], a in [0,p+1]^D
template <int D, class T>
__global__ void k_restrict(const T *__restrict__ R1, int p, int n1f, int n1c, const T *__restrict__ df,
                           T *__restrict__ dc) {
    const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nc = (D == 3) ? int64_t(n1c) * n1c * n1c : int64_t(n1c) * n1c;
    if (I >= nc) return;
    const int Ix = int(I % n1c), Iy = int((I / n1c) % n1c), Iz = (D == 3) ? int(I / (int64_t(n1c) * n1c)) : 0;
    const int w = p + 2;
    T acc = T(0);
    for (int az = 0; az < ((D == 3) ? w : 1); ++az) {
        const int jz = (D == 3) ? Iz - 1 + az : 0;
        if (D == 3 && (jz < 0 || jz >= n1f)) continue;
        const T rz = (D == 3) ? R1[Iz * w + az] : T(1);
        for (int ay = 0; ay < w; ++ay) {
            const int jy = Iy - 1 + ay;
            if (jy < 0 || jy >= n1f) continue;
            const T ry = R1[Iy * w + ay] * rz;
            T line = T(0);
            for (int ax = 0; ax < w; ++ax) {
                const int jx = Ix - 1 + ax;
                if (jx < 0 || jx >= n1f) continue;
                line += R1[Ix * w + ax] * df[(int64_t(jz) * n1f + jy) * n1f + jx];
            }
            acc += ry * line;
        }
    }
    dc[I] = acc;
}

// (P e_c)[i] = sum over coarse I with i - I + 1 in [0,p+1] per direction of
// R1[Ix][ix-Ix+1] R1[Iy][iy-Iy+1] (..) e_c[I]: the exact transpose of k_restrict.
template <int D, class T>
__device__ __forceinline__ T prolong_value(const T *__restrict__ R1, int p, int n1f, int n1c,
                                           const T *__restrict__ ec, int ix, int iy, int iz) {
    const int w = p + 2;
    T acc = T(0);
    for (int Iz = ((D == 3) ? iz - p : 0); Iz <= ((D == 3) ? iz + 1 : 0); ++Iz) {
        if (D == 3 && (Iz < 0 || Iz >= n1c)) continue;
        const T rz = (D == 3) ? R1[Iz * w + (iz - Iz + 1)] : T(1);
        for (int Iy = iy - p; Iy <= iy + 1; ++Iy) {
            if (Iy < 0 || Iy >= n1c) continue;
            const T ry = R1[Iy * w + (iy - Iy + 1)] * rz;
            T line = T(0);
            for (int Ix = ix - p; Ix <= ix + 1; ++Ix) {
                if (Ix < 0 || Ix >= n1c) continue;
                line += R1[Ix * w + (ix - Ix + 1)] * ec[(int64_t(Iz) * n1c + Iy) * n1c + Ix];
            }
            acc += ry * line;
        }
    }
    return acc;
}

template <int D, class T>
__global__ void k_prolong_add(const T *__restrict__ R1, int p, int n1f, int n1c, const T *__restrict__ ec,
                              T *__restrict__ uf) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nf = (D == 3) ? int64_t(n1f) * n1f * n1f : int64_t(n1f) * n1f;
    if (i >= nf) return;
    const int ix = int(i % n1f), iy = int((i / n1f) % n1f), iz = (D == 3) ? int(i / (int64_t(n1f) * n1f)) : 0;
    uf[i] += prolong_value<D, T>(R1, p, n1f, n1c, ec, ix, iy, iz);
}

// u64 += sigma * (e + P e_c): end of a correction cycle
template <int D, class T>
__global__ void k_prolong_update(const T *__restrict__ R1, int p, int n1f, int n1c, const T *__restrict__ ec,
                                 const T *__restrict__ e, double *__restrict__ u, const double *__restrict__ scal,
                                 int scaled) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nf = (D == 3) ? int64_t(n1f) * n1f * n1f : int64_t(n1f) * n1f;
    if (i >= nf) return;
    const int ix = int(i % n1f), iy = int((i / n1f) % n1f), iz = (D == 3) ? int(i / (int64_t(n1f) * n1f)) : 0;
    const T corr = e[i] + prolong_value<D, T>(R1, p, n1f, n1c, ec, ix, iy, iz);
    u[i] += scaled ? scal[kScalSigma] * double(corr) : double(corr);
}

// --------------------------------------------------------------- V-cycle --
// Red-black half step on a level: points of the given colour (parity of the
// index sum) are updated from e_src, the others copied; e_dst != e_src.
template <int D, class T>
__global__ void k_rb_half(const T *__restrict__ S, int n1, int colour, const T *__restrict__ e_src,
                          const T *__restrict__ rhs, T *__restrict__ e_dst, int zero_src) {
    const int64_t n = (D == 3) ? int64_t(n1) * n1 * n1 : int64_t(n1) * n1;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ix = int(i % n1), iy = int((i / n1) % n1), iz = (D == 3) ? int(i / (int64_t(n1) * n1)) : 0;
    const T ei = zero_src ? T(0) : e_src[i];
    if (((ix + iy + iz) & 1) != colour) {
        e_dst[i] = ei;
        return;
    }
    constexpr int W3 = (D == 3) ? 27 : 9;
    constexpr int c0 = (W3 - 1) / 2;
    T acc = T(0);
    if (!zero_src) {
        int w = 0;
        for (int oz = ((D == 3) ? -1 : 0); oz <= ((D == 3) ? 1 : 0); ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox, ++w) {
                    const int jx = ix + ox, jy = iy + oy, jz = iz + oz;
                    if (jx < 0 || jx >= n1 || jy < 0 || jy >= n1 || (D == 3 && (jz < 0 || jz >= n1))) continue;
                    acc += S[int64_t(w) * n + i] * e_src[(int64_t(jz) * n1 + jy) * n1 + jx];
                }
    }
    e_dst[i] = ei + (rhs[i] - acc) / S[int64_t(c0) * n + i];
}

// rc = P^T (rhs - S e) with P the linear interpolation onto odd fine indices
template <int D, class T>
__global__ void k_res_restrict(const T *__restrict__ S, int n1f, const T *__restrict__ e, const T *__restrict__ rhs,
                               int n1c, T *__restrict__ rc) {
    const int64_t nc = (D == 3) ? int64_t(n1c) * n1c * n1c : int64_t(n1c) * n1c;
    const int64_t nf = (D == 3) ? int64_t(n1f) * n1f * n1f : int64_t(n1f) * n1f;
    const int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    const int Ix = int(I % n1c), Iy = int((I / n1c) % n1c), Iz = (D == 3) ? int(I / (int64_t(n1c) * n1c)) : 0;
    T acc = T(0);
    for (int az = ((D == 3) ? -1 : 0); az <= ((D == 3) ? 1 : 0); ++az) {
        const int iz = (D == 3) ? 2 * Iz + 1 + az : 0;
        if (D == 3 && iz >= n1f) continue;
        const T wz = (D == 3) ? (az == 0 ? T(1) : T(0.5)) : T(1);
        for (int ay = -1; ay <= 1; ++ay) {
            const int iy = 2 * Iy + 1 + ay;
            if (iy >= n1f) continue;
            const T wy = (ay == 0 ? T(1) : T(0.5)) * wz;
            for (int ax = -1; ax <= 1; ++ax) {
                const int ix = 2 * Ix + 1 + ax;
                if (ix >= n1f) continue;
                const T wxy = (ax == 0 ? T(1) : T(0.5)) * wy;
                const int64_t i = (int64_t(iz) * n1f + iy) * n1f + ix;
                T s = T(0);
                int w = 0;
                for (int oz = ((D == 3) ? -1 : 0); oz <= ((D == 3) ? 1 : 0); ++oz)
                    for (int oy = -1; oy <= 1; ++oy)
                        for (int ox = -1; ox <= 1; ++ox, ++w) {
                            const int jx = ix + ox, jy = iy + oy, jz = iz + oz;
                            if (jx < 0 || jx >= n1f || jy < 0 || jy >= n1f || (D == 3 && (jz < 0 || jz >= n1f)))
                                continue;
                            s += S[int64_t(w) * nf + i] * e[(int64_t(jz) * n1f + jy) * n1f + jx];
                        }
                acc += wxy * (rhs[i] - s);
            }
        }
    }
    rc[I] = acc;
}

// e += P e_c
template <int D, class T>
__global__ void k_interp_add(const T *__restrict__ ec, int n1c, T *__restrict__ e, int n1f) {
    const int64_t nf = (D == 3) ? int64_t(n1f) * n1f * n1f : int64_t(n1f) * n1f;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int ix = int(i % n1f), iy = int((i / n1f) % n1f), iz = (D == 3) ? int(i / (int64_t(n1f) * n1f)) : 0;
    int Ix[2], Iy[2], Iz[2];
    T wx[2], wy[2], wz[2];
    int nx = 0, ny = 0, nz = 0;
    auto parents = [n1c](int v, int *I, T *w) {
        int c = 0;
        if (v & 1) {
            I[c] = (v - 1) / 2; w[c++] = T(1);
        } else {
            if (v / 2 - 1 >= 0) { I[c] = v / 2 - 1; w[c++] = T(0.5); }
            if (v / 2 < n1c) { I[c] = v / 2; w[c++] = T(0.5); }
        }
        return c;
    };
    nx = parents(ix, Ix, wx);
    ny = parents(iy, Iy, wy);
    if (D == 3) nz = parents(iz, Iz, wz);
    else { nz = 1; Iz[0] = 0; wz[0] = T(1); }
    T acc = T(0);
    for (int c = 0; c < nz; ++c)
        for (int b = 0; b < ny; ++b)
            for (int a = 0; a < nx; ++a)
                acc += wz[c] * wy[b] * wx[a] * ec[(int64_t(Iz[c]) * n1c + Iy[b]) * n1c + Ix[a]];
    e[i] += acc;
}

template <class T>
__global__ void k_coarsest(const T *__restrict__ rhs, T *__restrict__ e, double diag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) e[0] = rhs[0] / T(diag);
}

template <class T>
__global__ void k_fill_zero(T *__restrict__ x, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) x[i] = T(0);
}

template <class T>
__global__ void k_copy(const T *__restrict__ a, T *__restrict__ b, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// ----------------------------------------------------------------- DST --
// out[.., k, ..] = sum_i S[k][i] in[.., i, ..] along one axis (S symmetric);
// with mu != nullptr the result is divided by mu (diagonal solve).
__global__ void k_dst_axis(const double *__restrict__ S, int n1, int dim, int axis, const double *__restrict__ in,
                           double *__restrict__ out, const double *__restrict__ mu) {
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

template <class A, class B>
__global__ void k_convert(const A *__restrict__ a, B *__restrict__ b, int64_t n) {
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

template <class T>
const T *R1_of(const Problem &P) {
    return std::is_same<T, double>::value ? reinterpret_cast<const T *>(P.R1d64.ptr)
                                          : reinterpret_cast<const T *>(P.R1d32.ptr);
}

template <class T>
const T *S_of(const Level &L) {
    return std::is_same<T, double>::value ? reinterpret_cast<const T *>(L.S64.ptr)
                                          : reinterpret_cast<const T *>(L.S32.ptr);
}

template <class T>
void fill_zero(T *x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((k_fill_zero<T>), dim3(nblocks(n, 256)), dim3(256), 0, s, x, n);
}

// one V(nu1,nu2) cycle from zero on level l; result in e_out
template <class T>
void vcycle_level(Problem &P, size_t l, const T *rhs, T *e_out, int nu1, int nu2, hipStream_t s) {
    Level &L = P.levels[l];
    const int64_t n = L.g.n;
    const int d = P.dim;
    if (l + 1 == P.levels.size()) {
        hipLaunchKernelGGL((k_coarsest<T>), dim3(1), dim3(64), 0, s, rhs, e_out, L.coarsest_diag);
        return;
    }
    Level &C = P.levels[l + 1];
    T *buf[2] = {L.e[0].as<T>(), L.e[1].as<T>()};
    int cur = 0;
    bool zero = true;
    auto half = [&](int colour) {
        if (d == 2)
            hipLaunchKernelGGL((k_rb_half<2, T>), dim3(nblocks(n, 256)), dim3(256), 0, s, S_of<T>(L), L.g.n1, colour,
                               buf[cur], rhs, buf[1 - cur], zero ? 1 : 0);
        else
            hipLaunchKernelGGL((k_rb_half<3, T>), dim3(nblocks(n, 256)), dim3(256), 0, s, S_of<T>(L), L.g.n1, colour,
                               buf[cur], rhs, buf[1 - cur], zero ? 1 : 0);
        cur = 1 - cur;
        zero = false;
    };
    for (int k = 0; k < nu1; ++k) {
        half(0);
        half(1);
    }
    if (zero) {
        fill_zero(buf[cur], n, s);
        zero = false;
    }
    T *rc = C.rhs.as<T>();
    T *ecl = C.res.as<T>();
    if (d == 2)
        hipLaunchKernelGGL((k_res_restrict<2, T>), dim3(nblocks(C.g.n, 256)), dim3(256), 0, s, S_of<T>(L), L.g.n1,
                           buf[cur], rhs, C.g.n1, rc);
    else
        hipLaunchKernelGGL((k_res_restrict<3, T>), dim3(nblocks(C.g.n, 256)), dim3(256), 0, s, S_of<T>(L), L.g.n1,
                           buf[cur], rhs, C.g.n1, rc);
    vcycle_level<T>(P, l + 1, rc, ecl, nu1, nu2, s);
    if (d == 2)
        hipLaunchKernelGGL((k_interp_add<2, T>), dim3(nblocks(n, 256)), dim3(256), 0, s, ecl, C.g.n1, buf[cur], L.g.n1);
    else
        hipLaunchKernelGGL((k_interp_add<3, T>), dim3(nblocks(n, 256)), dim3(256), 0, s, ecl, C.g.n1, buf[cur], L.g.n1);
    for (int k = 0; k < nu2; ++k) {
        half(0);
        half(1);
    }
    hipLaunchKernelGGL((k_copy<T>), dim3(nblocks(n, 256)), dim3(256), 0, s, buf[cur], e_out, n);
}

}  // namespace

// ------------------------------------------------------------ launchers --
template <class T>
void launch_restrict(const Problem &P, const T *df, T *dc, hipStream_t s) {
    const int64_t nc = P.coarse.n;
    if (P.dim == 2)
        hipLaunchKernelGGL((k_restrict<2, T>), dim3(nblocks(nc, 256)), dim3(256), 0, s, R1_of<T>(P), P.p, P.fine.n1,
                           P.coarse.n1, df, dc);
    else
        hipLaunchKernelGGL((k_restrict<3, T>), dim3(nblocks(nc, 256)), dim3(256), 0, s, R1_of<T>(P), P.p, P.fine.n1,
                           P.coarse.n1, df, dc);
}
template void launch_restrict<double>(const Problem &, const double *, double *, hipStream_t);
template void launch_restrict<float>(const Problem &, const float *, float *, hipStream_t);

template <class T>
void launch_prolong_add(const Problem &P, const T *ec, T *uf, hipStream_t s) {
    const int64_t nf = P.fine.n;
    if (P.dim == 2)
        hipLaunchKernelGGL((k_prolong_add<2, T>), dim3(nblocks(nf, 256)), dim3(256), 0, s, R1_of<T>(P), P.p, P.fine.n1,
                           P.coarse.n1, ec, uf);
    else
        hipLaunchKernelGGL((k_prolong_add<3, T>), dim3(nblocks(nf, 256)), dim3(256), 0, s, R1_of<T>(P), P.p, P.fine.n1,
                           P.coarse.n1, ec, uf);
}
template void launch_prolong_add<double>(const Problem &, const double *, double *, hipStream_t);
template void launch_prolong_add<float>(const Problem &, const float *, float *, hipStream_t);

template <class T>
void launch_prolong_update(const Problem &P, const T *ec, const T *e, double *u, bool scaled, hipStream_t s) {
    const int64_t nf = P.fine.n;
    if (P.dim == 2)
        hipLaunchKernelGGL((k_prolong_update<2, T>), dim3(nblocks(nf, 256)), dim3(256), 0, s, R1_of<T>(P), P.p,
                           P.fine.n1, P.coarse.n1, ec, e, u, P.scal.as<double>(), scaled ? 1 : 0);
    else
        hipLaunchKernelGGL((k_prolong_update<3, T>), dim3(nblocks(nf, 256)), dim3(256), 0, s, R1_of<T>(P), P.p,
                           P.fine.n1, P.coarse.n1, ec, e, u, P.scal.as<double>(), scaled ? 1 : 0);
}
template void launch_prolong_update<double>(const Problem &, const double *, const double *, double *, bool,
                                            hipStream_t);
template void launch_prolong_update<float>(const Problem &, const float *, const float *, double *, bool,
                                           hipStream_t);

template <class T>
void launch_vcycle(Problem &P, const T *rhs, T *e, int nu1, int nu2, hipStream_t s) {
    IGA2L_REQUIRE(P.vcycle_ready, IGA2L_EINVAL, "V-cycle hierarchy not set up");
    vcycle_level<T>(P, 0, rhs, e, nu1, nu2, s);
}
template void launch_vcycle<double>(Problem &, const double *, double *, int, int, hipStream_t);
template void launch_vcycle<float>(Problem &, const float *, float *, int, int, hipStream_t);

void launch_dst_solve(Problem &P, const double *d, double *e, hipStream_t s) {
    IGA2L_REQUIRE(P.direct_ready, IGA2L_EINVAL, "exact coarse solver not set up");
    const int n1 = P.coarse.n1, dim = P.dim;
    const int64_t n = P.coarse.n;
    double *t1 = P.ctmp.as<double>();
    const double *S = P.dst_S.as<double>(), *mu = P.dst_mu.as<double>();
    // forward transform along every axis, diagonal solve, inverse (= forward) transform
    const double *src = d;
    double *bufs[2] = {t1, e};
    int cur = 0;
    for (int ax = 0; ax < dim; ++ax) {
        hipLaunchKernelGGL(k_dst_axis, dim3(nblocks(n, 256)), dim3(256), 0, s, S, n1, dim, ax, src, bufs[cur],
                           (ax == dim - 1) ? mu : nullptr);
        src = bufs[cur];
        cur = 1 - cur;
    }
    for (int ax = 0; ax < dim; ++ax) {
        hipLaunchKernelGGL(k_dst_axis, dim3(nblocks(n, 256)), dim3(256), 0, s, S, n1, dim, ax, src, bufs[cur],
                           nullptr);
        src = bufs[cur];
        cur = 1 - cur;
    }
    // 2*dim passes alternate t1, e, t1, e, ...: an even count, so the last one wrote e
}

void launch_convert(const void *src, void *dst, int64_t n, bool to_fp32, hipStream_t s) {
    if (to_fp32)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(nblocks(n, 256)), dim3(256), 0, s,
                           static_cast<const double *>(src), static_cast<float *>(dst), n);
    else
        hipLaunchKernelGGL((k_convert<float, double>), dim3(nblocks(n, 256)), dim3(256), 0, s,
                           static_cast<const float *>(src), static_cast<double *>(dst), n);
}

void launch_grad_kappa(const Problem &P, const double *u, const double *lam, double *g, hipStream_t s) {
    if (P.dim == 2)
        hipLaunchKernelGGL((k_grad_kappa<2>), dim3(nblocks(P.ne, 128)), dim3(128), 0, s, P.Ke_d.as<double>(), P.p, P.m,
                           P.fine.n1, u, lam, g);
    else
        hipLaunchKernelGGL((k_grad_kappa<3>), dim3(nblocks(P.ne, 128)), dim3(128), 0, s, P.Ke_d.as<double>(), P.p, P.m,
                           P.fine.n1, u, lam, g);
}

}  // namespace iga2l
