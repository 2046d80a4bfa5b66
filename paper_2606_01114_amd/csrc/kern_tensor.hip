// Demag tensor setup on the GPU in FP64: the real-space octant (Newell's
// closed form near, moment-matched dipole quadrature far), and the final
// scaling/permutation of its real spectrum into the layout of the fused pass.
// Also the element-wise kernels of the RK4 adjoint.
#include "passes.hpp"
#include "kernels.hpp"
#include <algorithm>

namespace mmx {

// Newell's f: even in every argument
__device__ double newell_f(double x, double y, double z) {
    x = fabs(x); y = fabs(y); z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double r = 0.0, p;
    p = y * (z2 - x2) * 0.5;
    if (p != 0.0) r += p * asinh(y / sqrt(x2 + z2));
    p = z * (y2 - x2) * 0.5;
    if (p != 0.0) r += p * asinh(z / sqrt(x2 + y2));
    p = x * y * z;
    if (p != 0.0) r -= p * atan(y * z / (x * R));
    r += (2.0 * x2 - y2 - z2) * R * (1.0 / 6.0);
    return r;
}

// Newell's g: odd in x and y, even in z
__device__ double newell_g(double x, double y, double z) {
    if (x == 0.0 || y == 0.0) return 0.0;
    const double s = ((x < 0.0) != (y < 0.0)) ? -1.0 : 1.0;
    x = fabs(x); y = fabs(y); z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double r = 0.0, p;
    p = x * y * z;
    if (p != 0.0) r += p * asinh(z / sqrt(x2 + y2));
    p = y * (3.0 * z2 - y2) * (1.0 / 6.0);
    if (p != 0.0) r += p * asinh(x / sqrt(y2 + z2));
    p = x * (3.0 * z2 - x2) * (1.0 / 6.0);
    if (p != 0.0) r += p * asinh(y / sqrt(x2 + z2));
    p = z * z2 * (1.0 / 6.0);
    if (p != 0.0) r -= p * atan(x * y / (z * R));
    p = z * y2 * 0.5;
    if (p != 0.0) r -= p * atan(x * z / (y * R));
    p = z * x2 * 0.5;
    if (p != 0.0) r -= p * atan(y * z / (x * R));
    r -= x * y * R * (1.0 / 3.0);
    return s * r;
}

template <bool G>
__device__ double stencil27(double X, double Y, double Z, double a, double b, double c) {
    double acc = 0.0;
    for (int e1 = -1; e1 <= 1; ++e1)
        for (int e2 = -1; e2 <= 1; ++e2)
            for (int e3 = -1; e3 <= 1; ++e3) {
                const double w = (double)((e1 == 0 ? 2 : -1) * (e2 == 0 ? 2 : -1) * (e3 == 0 ? 2 : -1));
                const double x = X + e1 * a, y = Y + e2 * b, z = Z + e3 * c;
                acc += w * (G ? newell_g(x, y, z) : newell_f(x, y, z));
            }
    return acc;
}

__device__ void tensor_at(int64_t i, int64_t j, int64_t k, double dx, double dy, double dz, double P, double out[6]) {
    const double X = (double)i * dx, Y = (double)j * dy, Z = (double)k * dz;
    const double dmax = fmax(dx, fmax(dy, dz));
    const double r2 = X * X + Y * Y + Z * Z, lim = P * dmax;
    if (P <= 0.0 || r2 <= lim * lim) {
        const double norm = 1.0 / (4.0 * M_PI * dx * dy * dz);
        out[0] = stencil27<false>(X, Y, Z, dx, dy, dz) * norm;
        out[1] = stencil27<false>(Y, X, Z, dy, dx, dz) * norm;
        out[2] = stencil27<false>(Z, Y, X, dz, dy, dx) * norm;
        out[3] = stencil27<true>(X, Y, Z, dx, dy, dz) * norm;
        out[4] = stencil27<true>(X, Z, Y, dx, dz, dy) * norm;
        out[5] = stencil27<true>(Y, Z, X, dy, dz, dx) * norm;
    } else {
        const double s = 0.63245553203367586639977870888654371;  // sqrt(2/5)
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int e1 = -1; e1 <= 1; ++e1)
            for (int e2 = -1; e2 <= 1; ++e2)
                for (int e3 = -1; e3 <= 1; ++e3) {
                    const double w = (e1 == 0 ? 7.0 / 12.0 : 5.0 / 24.0) * (e2 == 0 ? 7.0 / 12.0 : 5.0 / 24.0) *
                                     (e3 == 0 ? 7.0 / 12.0 : 5.0 / 24.0);
                    const double x = ((double)i + e1 * s) * dx, y = ((double)j + e2 * s) * dy,
                                 z = ((double)k + e3 * s) * dz;
                    const double rr = x * x + y * y + z * z;
                    const double q = w / (rr * rr * sqrt(rr));
                    acc[0] += q * (rr - 3.0 * x * x);
                    acc[1] += q * (rr - 3.0 * y * y);
                    acc[2] += q * (rr - 3.0 * z * z);
                    acc[3] += q * (-3.0 * x * y);
                    acc[4] += q * (-3.0 * x * z);
                    acc[5] += q * (-3.0 * y * z);
                }
        const double pref = dx * dy * dz / (4.0 * M_PI);
        for (int q = 0; q < 6; ++q) out[q] = acc[q] * pref;
    }
    // an odd component is exactly zero where its odd-axis offset is zero
    if (i == 0 || j == 0) out[3] = 0.0;
    if (i == 0 || k == 0) out[4] = 0.0;
    if (j == 0 || k == 0) out[5] = 0.0;
}

__global__ void __launch_bounds__(256) k_tensor_octant(double *out, int nx, int ny, int nz, double dx, double dy,
                                                        double dz, double P) {
    const int64_t total = (int64_t)nx * ny * nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int64_t k = t % nz, ij = t / nz;
    const int64_t j = ij % ny, i = ij / ny;
    double v[6];
    tensor_at(i, j, k, dx, dy, dz, P, v);
    for (int q = 0; q < 6; ++q) out[t * 6 + q] = v[q];
}

// [kx'][ky'][kz][6] FP64 -> [kz][kx'][ky'][6] in T, scaled: the stored value is
// -N^/(Lx Ly Lz); the separable cosine/sine transforms drop a factor (-i) per
// odd axis, i.e. -1 for the off-diagonal components.
template <typename T>
__global__ void __launch_bounds__(256) k_tensor_finalize(const double *__restrict__ in, T *__restrict__ out, int hx,
                                                          int hy, int hz, double inv_ltot) {
    const int64_t total = (int64_t)hx * hy * hz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int64_t kz = t % hz, r = t / hz;
    const int64_t ky = r % hy, kx = r / hy;
    const double *src = in + t * 6;
    T *dst = out + (((kz * hx + kx) * hy) + ky) * 6;
    for (int q = 0; q < 6; ++q) dst[q] = T((q < 3 ? -src[q] : src[q]) * inv_ltot);
}

// inverse permutation (test hook): [kz][kx'][ky'][6] T -> [kx'][ky'][kz][6] double
template <typename T>
__global__ void __launch_bounds__(256) k_tensor_export(const T *__restrict__ in, double *__restrict__ out, int hx,
                                                        int hy, int hz) {
    const int64_t total = (int64_t)hx * hy * hz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int64_t kz = t % hz, r = t / hz;
    const int64_t ky = r % hy, kx = r / hy;
    const T *src = in + (((kz * hx + kx) * hy) + ky) * 6;
    for (int q = 0; q < 6; ++q) out[t * 6 + q] = (double)src[q];
}

// RK4 adjoint, element-wise: u_bar = (I - u^ u^T) g / |u| (or g), also copied
// into the running cotangent of m.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_unorm(const T *__restrict__ g, const T *__restrict__ u, T *__restrict__ ub,
                                                    T *__restrict__ gsum, int renorm, int64_t ncell) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncell) return;
    T gv[3] = {g[3 * t], g[3 * t + 1], g[3 * t + 2]};
    T o[3];
    if (renorm) {
        const T u0 = u[3 * t], u1 = u[3 * t + 1], u2 = u[3 * t + 2];
        const T nu = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
        const T h0 = u0 / nu, h1 = u1 / nu, h2 = u2 / nu;
        const T d = h0 * gv[0] + h1 * gv[1] + h2 * gv[2];
        o[0] = (gv[0] - h0 * d) / nu;
        o[1] = (gv[1] - h1 * d) / nu;
        o[2] = (gv[2] - h2 * d) / nu;
    } else {
        o[0] = gv[0]; o[1] = gv[1]; o[2] = gv[2];
    }
    for (int c = 0; c < 3; ++c) { ub[3 * t + c] = o[c]; gsum[3 * t + c] = o[c]; }
}

// s_bar = ym + gmh; gsum += s_bar; kb = w * ub + coef * s_bar (if kb)
template <typename T>
__global__ void __launch_bounds__(256) k_adj_combine(const T *__restrict__ ym, const T *__restrict__ gmh,
                                                      const T *__restrict__ ub, T *__restrict__ gsum, T *__restrict__ kb,
                                                      double w, double coef, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const T sb = ym[t] + gmh[t];
    gsum[t] = gsum[t] + sb;
    if (kb) kb[t] = T(w) * ub[t] + T(coef) * sb;
}

template <typename T>
__global__ void __launch_bounds__(256) k_scale_copy(const T *__restrict__ in, T *__restrict__ out, double s, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    out[t] = T(s) * in[t];
}

// plain streaming copy, 16 bytes per lane per iteration
__global__ void __launch_bounds__(256) k_copy16(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_tensor_octant(double *out, int nx, int ny, int nz, double dx, double dy, double dz, double P,
                                hipStream_t s) {
    const int64_t total = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL(k_tensor_octant, dim3(nblk(total, 256)), dim3(256), 0, s, out, nx, ny, nz, dx, dy, dz, P);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tensor_finalize(const double *in, T *out, int hx, int hy, int hz, double inv_ltot, hipStream_t s) {
    const int64_t total = (int64_t)hx * hy * hz;
    hipLaunchKernelGGL((k_tensor_finalize<T>), dim3(nblk(total, 256)), dim3(256), 0, s, in, out, hx, hy, hz, inv_ltot);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tensor_export(const T *in, double *out, int hx, int hy, int hz, hipStream_t s) {
    const int64_t total = (int64_t)hx * hy * hz;
    hipLaunchKernelGGL((k_tensor_export<T>), dim3(nblk(total, 256)), dim3(256), 0, s, in, out, hx, hy, hz);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_unorm(const T *g, const T *u, T *ub, T *gsum, int renorm, int64_t ncell, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_unorm<T>), dim3(nblk(ncell, 256)), dim3(256), 0, s, g, u, ub, gsum, renorm, ncell);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_combine(const T *ym, const T *gmh, const T *ub, T *gsum, T *kb, double w, double coef, int64_t n,
                              hipStream_t s) {
    hipLaunchKernelGGL((k_adj_combine<T>), dim3(nblk(n, 256)), dim3(256), 0, s, ym, gmh, ub, gsum, kb, w, coef, n);
    return hipGetLastError();
}

hipError_t launch_copy16(const void *src, void *dst, int64_t n16, hipStream_t s) {
    if (n16 <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 1024);
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (const float4 *)src, (float4 *)dst, n16);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_copy(const T *in, T *out, double s, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_scale_copy<T>), dim3(nblk(n, 256)), dim3(256), 0, st, in, out, s, n);
    return hipGetLastError();
}

template hipError_t launch_scale_copy<float>(const float *, float *, double, int64_t, hipStream_t);
template hipError_t launch_scale_copy<double>(const double *, double *, double, int64_t, hipStream_t);
template hipError_t launch_tensor_finalize<float>(const double *, float *, int, int, int, double, hipStream_t);
template hipError_t launch_tensor_finalize<double>(const double *, double *, int, int, int, double, hipStream_t);
template hipError_t launch_tensor_export<float>(const float *, double *, int, int, int, hipStream_t);
template hipError_t launch_tensor_export<double>(const double *, double *, int, int, int, hipStream_t);
template hipError_t launch_adj_unorm<float>(const float *, const float *, float *, float *, int, int64_t, hipStream_t);
template hipError_t launch_adj_unorm<double>(const double *, const double *, double *, double *, int, int64_t, hipStream_t);
template hipError_t launch_adj_combine<float>(const float *, const float *, const float *, float *, float *, double,
                                              double, int64_t, hipStream_t);
template hipError_t launch_adj_combine<double>(const double *, const double *, const double *, double *, double *,
                                               double, double, int64_t, hipStream_t);

}  // namespace mmx
