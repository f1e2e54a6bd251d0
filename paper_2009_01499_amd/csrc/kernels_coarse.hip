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
// d_c[I] = sum_a R1[Ix][ax] R1[Iy][ay] (R1[Iz][az]) d[I - 1 + a], a in [0,p+1]^D
template <int D, class T>
__global__ void k_restrict(const T *__restrict__ R1, int p, int n1f, int n1c, const T *__restrict__ df,
                           T *__restrict__ dc, const int *__restrict__ skip) {
    const int stop = skip ? *skip : 0;  // tested before the store (hides the load latency)
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
    if (stop) return;
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
                              T *__restrict__ uf, const int *__restrict__ skip) {
    if (skip && *skip) return;
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
                                 int scaled, const int *__restrict__ skip) {
    const int stop = skip ? *skip : 0;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nf = (D == 3) ? int64_t(n1f) * n1f * n1f : int64_t(n1f) * n1f;
    if (i >= nf) return;
    const int ix = int(i % n1f), iy = int((i / n1f) % n1f), iz = (D == 3) ? int(i / (int64_t(n1f) * n1f)) : 0;
    const T corr = e[i] + prolong_value<D, T>(R1, p, n1f, n1c, ec, ix, iy, iz);
    if (stop) return;
    u[i] += scaled ? scal[kScalSigma] * double(corr) : double(corr);
}

// ----------------------------------------------------------------- DST --
// out[.., k, ..] = sum_i S[k][i] in[.., i, ..] along one axis (S symmetric);
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

template <class T>
const T *R1_of(const Problem &P) {
    return std::is_same<T, double>::value ? reinterpret_cast<const T *>(P.R1d64.ptr)
                                          : reinterpret_cast<const T *>(P.R1d32.ptr);
}

}  // namespace

// ------------------------------------------------------------ launchers --
template <class T>
void launch_restrict(const Problem &P, const T *df, T *dc, hipStream_t s) {
    if (P.dim == 2) {
        launch_restrict2d<T>(P, df, dc, s);
        return;
    }
    const int64_t nc = P.coarse.n;
    hipLaunchKernelGGL((k_restrict<3, T>), dim3(nblocks(nc, 256)), dim3(256), 0, s, R1_of<T>(P), P.p, P.fine.n1,
                       P.coarse.n1, df, dc, P.skip);
}
template void launch_restrict<double>(const Problem &, const double *, double *, hipStream_t);
template void launch_restrict<float>(const Problem &, const float *, float *, hipStream_t);

template <class T>
void launch_prolong_add(const Problem &P, const T *ec, T *uf, hipStream_t s) {
    if (P.dim == 2) {
        launch_prolong2d<T>(P, ec, uf, nullptr, nullptr, false, s);
        return;
    }
    const int64_t nf = P.fine.n;
    hipLaunchKernelGGL((k_prolong_add<3, T>), dim3(nblocks(nf, 256)), dim3(256), 0, s, R1_of<T>(P), P.p, P.fine.n1,
                       P.coarse.n1, ec, uf, P.skip);
}
template void launch_prolong_add<double>(const Problem &, const double *, double *, hipStream_t);
template void launch_prolong_add<float>(const Problem &, const float *, float *, hipStream_t);

template <class T>
void launch_prolong_update(const Problem &P, const T *ec, const T *e, double *u, bool scaled, hipStream_t s) {
    if (P.dim == 2) {
        launch_prolong2d<T>(P, ec, nullptr, e, u, scaled, s);
        return;
    }
    const int64_t nf = P.fine.n;
    hipLaunchKernelGGL((k_prolong_update<3, T>), dim3(nblocks(nf, 256)), dim3(256), 0, s, R1_of<T>(P), P.p,
                       P.fine.n1, P.coarse.n1, ec, e, u, P.scal.as<double>(), scaled ? 1 : 0, P.skip);
}
template void launch_prolong_update<double>(const Problem &, const double *, const double *, double *, bool,
                                            hipStream_t);
template void launch_prolong_update<float>(const Problem &, const float *, const float *, double *, bool,
                                           hipStream_t);

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
                           (ax == dim - 1) ? mu : nullptr, P.skip);
        src = bufs[cur];
        cur = 1 - cur;
    }
    for (int ax = 0; ax < dim; ++ax) {
        hipLaunchKernelGGL(k_dst_axis, dim3(nblocks(n, 256)), dim3(256), 0, s, S, n1, dim, ax, src, bufs[cur],
                           nullptr, P.skip);
        src = bufs[cur];
        cur = 1 - cur;
    }
    // 2*dim passes alternate t1, e, t1, e, ...: an even count, so the last one wrote e
}

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

}  // namespace iga2l
