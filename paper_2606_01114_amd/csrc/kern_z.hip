// The z passes: forward real-to-complex along z (first pass of the
// convolution, source = Ms m, or a cotangent) and the inverse complex-to-real
// along z fused with its epilogue (exchange stencil, h_eff output and FP64
// energy partials; or the LLG right-hand side and the RK4 stage update,
// followed by the forward z transform of the next stage's input; or the
// adjoint of h_eff).  Two real z-lines share one complex FFT.
#include "passes.hpp"
#include "kernels.hpp"
#include "zepi.hpp"

namespace mmx {

// zero the paired z-lines of a tile
template <typename T>
__device__ __forceinline__ void zero_lines(cplx<T> *lds, int nlc, int L, int pitch, int tid, int nthr) {
    const cplx<T> z = cmake<cplx<T>>(T(0), T(0));
    for (int e = tid; e < nlc * L; e += nthr) {
        const int u = e / L, k = e - u * L;
        lds[u * pitch + k] = z;
    }
}

// forward z transform of the LDS lines and the split of each complex line
// into the half spectra of its two real lines, written to S1 [kz][pos][c]
template <typename T>
__device__ __forceinline__ void zfwd_tail(cplx<T> *lds, const ZGeom &g, int64_t pos0, int wp, int tid, int ltid) {
    using C = cplx<T>;
    const int nlr = 3 * wp, nlc = (nlr + 1) / 2;
    lds_fft<T, -1>(lds, nlc, g.pitch, g.f, reinterpret_cast<const C *>(g.tw), ltid, g.nthr);
    if (tid < g.nthr) {
        const int64_t npos3 = (int64_t)g.nx * g.ny * 3;
        C *S1 = reinterpret_cast<C *>(g.S1) + pos0 * 3;
        const int L = g.Lz;
        const T half = T(0.5);
        const FastDiv dw = make_fastdiv((uint32_t)nlr);
        for (int e = tid; e < g.hz * nlr; e += g.nthr) {
            const int k = (int)fdiv((uint32_t)e, dw), l = e - k * nlr;
            const int u = l >> 1;
            const C zk = lds[u * g.pitch + k];
            const C zm = lds[u * g.pitch + (k == 0 ? 0 : L - k)];
            C v;
            if ((l & 1) == 0) v = cmake<C>(half * (zk.x + zm.x), half * (zk.y - zm.y));
            else v = cmake<C>(half * (zk.y + zm.y), -half * (zk.x - zm.x));
            S1[k * npos3 + l] = v;
        }
    }
}

template <typename T, int SRC>
__device__ __forceinline__ void zfwd_body(const ZFwdArgs &a, uint32_t tile) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const ZGeom &g = a.g;
    const int tid = threadIdx.x, ltid = tid < g.nthr ? tid : 1 << 30;
    const int64_t npos = (int64_t)g.nx * g.ny;
    const int64_t pos0 = (int64_t)tile * g.P;
    const int wp = (int)min((int64_t)g.P, npos - pos0);
    const int nlr = 3 * wp, nlc = (nlr + 1) / 2;
    if (tid < g.nthr) zero_lines<T>(lds, nlc, g.Lz, g.pitch, tid, g.nthr);
    __syncthreads();
    if (tid < g.nthr) {
        const int nz = g.nz;
        const int64_t cell0 = pos0 * nz;
        if (SRC != SRC_ADJPRE) {
            const T *src = reinterpret_cast<const T *>(a.src) + cell0 * 3;
            const T *Ms = reinterpret_cast<const T *>(a.Ms);
            const T Ms_s = T(a.Ms_scalar);
            const int nz3 = nz * 3;
            const FastDiv d3 = make_fastdiv((uint32_t)nz3);
            for (int e = tid; e < wp * nz3; e += g.nthr) {
                const int pl = (int)fdiv((uint32_t)e, d3), rem = e - pl * nz3;
                const int z = rem / 3, c = rem - z * 3;
                T v = src[e];
                if (SRC == SRC_MS_M) v *= ms_at(Ms, Ms_s, cell0 + (int64_t)pl * nz + z);
                const int l = pl * 3 + c;
                reinterpret_cast<T *>(&lds[(l >> 1) * g.pitch + z])[l & 1] = v;
            }
        } else {
            // y = VJP of f(s, h) = -g'[s x h + alpha s x (s x h)] for cotangent kb
            const T *s = reinterpret_cast<const T *>(a.s) + cell0 * 3;
            const T *h = reinterpret_cast<const T *>(a.h) + cell0 * 3;
            const T *kb = reinterpret_cast<const T *>(a.kb) + cell0 * 3;
            T *ym = reinterpret_cast<T *>(a.ym) + cell0 * 3;
            T *yh = reinterpret_cast<T *>(a.yh) + cell0 * 3;
            const T gp = T(a.gp), al = T(a.alpha);
            for (int e = tid; e < wp * nz; e += g.nthr) {
                const int pl = (int)fdiv((uint32_t)e, g.dnz), z = e - pl * nz;
                T sv[3], hv[3], y[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) { sv[c] = s[3 * e + c]; hv[c] = h[3 * e + c]; y[c] = kb[3 * e + c]; }
                T av[3], yxm[3], hxy[3], axy[3], hxyxm[3], yxmxm[3];
                cross3(sv, hv, av);
                cross3(y, sv, yxm);
                cross3(hv, y, hxy);
                cross3(av, y, axy);
                cross3(hv, yxm, hxyxm);
                cross3(yxm, sv, yxmxm);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T vm = -gp * (hxy[c] + al * (axy[c] + hxyxm[c]));
                    const T vh = -gp * (yxm[c] + al * yxmxm[c]);
                    ym[3 * e + c] = vm;
                    yh[3 * e + c] = vh;
                    const int l = pl * 3 + c;
                    reinterpret_cast<T *>(&lds[(l >> 1) * g.pitch + z])[l & 1] = vh;
                }
            }
        }
    }
    __syncthreads();
    zfwd_tail<T>(lds, g, pos0, wp, tid, ltid);
}

template <typename T, int EPI>
__device__ __forceinline__ void zinv_body(const ZInvArgs &a, uint32_t blk) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const ZGeom &g = a.g;
    const int tid = threadIdx.x, ltid = tid < g.nthr ? tid : 1 << 30;
    const int64_t npos = (int64_t)g.nx * g.ny;
    const int64_t pos0 = (int64_t)blk * g.P;
    const int wp = (int)min((int64_t)g.P, npos - pos0);
    const int nlr = 3 * wp, nlc = (nlr + 1) / 2;
    const int L = g.Lz, hz = g.hz, pitch = g.pitch;
    const bool demag = (a.terms & 1u) != 0, exch = (a.terms & 2u) != 0;
    // 1. Hermitian extension of the paired half spectra (S1 [kz][pos][c]:
    //    line l of this tile at kz sits at (kz*npos + pos0)*3 + l)
    if (demag && tid < g.nthr) {
        const int64_t npos3 = npos * 3;
        const C *S1 = reinterpret_cast<const C *>(g.S1) + pos0 * 3;
        const FastDiv dl = make_fastdiv((uint32_t)nlc);
        for (int e = tid; e < nlc * hz; e += g.nthr) {
            const int k = (int)fdiv((uint32_t)e, dl), u = e - k * nlc;
            const int l0 = 2 * u, l1 = 2 * u + 1;
            C A = cmake<C>(T(0), T(0)), B = A;
            A = S1[k * npos3 + l0];
            if (l1 < nlr) B = S1[k * npos3 + l1];
            if (k == 0 || 2 * k == L) {
                lds[u * pitch + k] = cmake<C>(A.x, B.x);
            } else {
                lds[u * pitch + k] = cmake<C>(A.x - B.y, A.y + B.x);
                lds[u * pitch + (L - k)] = cmake<C>(A.x + B.y, B.x - A.y);
            }
        }
    }
    __syncthreads();
    if (demag) lds_fft<T, +1>(lds, nlc, pitch, g.f, reinterpret_cast<const C *>(g.tw), ltid, g.nthr);
    // 2. epilogue per cell
    Acc4 acc;
    const int nz = g.nz, ny = g.ny;
    if (tid < g.nthr) {
        for (int e = tid; e < wp * nz; e += g.nthr) {
            const int pl = (int)fdiv((uint32_t)e, g.dnz), z = e - pl * nz;
            const int64_t pos = pos0 + pl;
            const int i = (int)fdiv((uint32_t)pos, g.dny), j = (int)(pos - (int64_t)i * ny);
            const int64_t cell = pos * nz + z;
            T hd[3] = {T(0), T(0), T(0)};
            if (demag) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int l = pl * 3 + c;
                    hd[c] = reinterpret_cast<const T *>(&lds[(l >> 1) * pitch + z])[l & 1];
                }
            }
            T src[3] = {T(0), T(0), T(0)};
            cell_epilogue<T, EPI>(a, cell, i, j, z, hd, acc, src);
            if ((EPI == EPI_STAGE || EPI == EPI_TAB) && a.next_r2c) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int l = pl * 3 + c;
                    reinterpret_cast<T *>(&lds[(l >> 1) * pitch + z])[l & 1] = src[c];
                }
            }
        }
    }
    if (EPI == EPI_HEFF && a.epart) block_energy(acc.v[0], acc.v[1], reinterpret_cast<double *>(smem), a.epart + 2 * (int64_t)blk, tid);
    if (EPI == EPI_TAB && a.tab_last) block_max(acc.v[0], reinterpret_cast<double *>(smem), a.epart + 2 * (int64_t)blk, tid);
    if (EPI == EPI_BB) block_bb(acc, reinterpret_cast<double *>(smem), a.bb_part + 4 * (int64_t)blk, tid);
    if ((EPI == EPI_STAGE || EPI == EPI_TAB) && a.next_r2c) {
        // zero the padding rows and the unused half of an odd last line, then
        // transform the next stage's source along z
        if (tid < g.nthr) {
            const C zc = cmake<C>(T(0), T(0));
            const int pad = L - nz;
            for (int e = tid; e < nlc * pad; e += g.nthr) {
                const int u = e / pad, k = nz + (e - u * pad);
                lds[u * pitch + k] = zc;
            }
            if (nlr & 1) {
                for (int k = tid; k < nz; k += g.nthr) reinterpret_cast<T *>(&lds[(nlc - 1) * pitch + k])[1] = T(0);
            }
        }
        __syncthreads();
        zfwd_tail<T>(lds, g, pos0, wp, tid, ltid);
    }
}

template <typename T, int SRC>
__global__ void __launch_bounds__(1024) k_zfwd(const ZFwdArgs a) { zfwd_body<T, SRC>(a, xcd_tile(blockIdx.x, gridDim.x)); }

template <typename T, int SRC>
__global__ void __launch_bounds__(1024) k_zfwd_b(const ZFwdArgs *__restrict__ d, const int2 *__restrict__ map) {
    const int2 e = map[xcd_tile(blockIdx.x, gridDim.x)];
    zfwd_body<T, SRC>(d[e.x], (uint32_t)e.y);
}

template <typename T, int EPI>
__global__ void __launch_bounds__(1024) k_zinv(const ZInvArgs a) { zinv_body<T, EPI>(a, xcd_tile(blockIdx.x, gridDim.x)); }

template <typename T, int EPI>
__global__ void __launch_bounds__(1024) k_zinv_b(const ZInvArgs *__restrict__ d, const int2 *__restrict__ map) {
    const int2 e = map[xcd_tile(blockIdx.x, gridDim.x)];
    zinv_body<T, EPI>(d[e.x], (uint32_t)e.y);
}

// deterministic final sum of the per-block energy partials (one block)
__global__ void __launch_bounds__(256) k_energy_reduce(const double *__restrict__ part, int nblk, double *out) {
    __shared__ double r0[256], r1[256];
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) { s0 += part[2 * b]; s1 += part[2 * b + 1]; }
    r0[threadIdx.x] = s0;
    r1[threadIdx.x] = s1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) { r0[threadIdx.x] += r0[threadIdx.x + w]; r1[threadIdx.x] += r1[threadIdx.x + w]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[0] = r0[0]; out[1] = r1[0]; }
}

template <typename T>
hipError_t launch_zfwd(const ZFwdArgs &a, int src_mode, size_t lds_bytes, hipStream_t s) {
    if (a.g.tiles <= 0) return hipSuccess;
    switch (src_mode) {
    case SRC_MS_M: hipLaunchKernelGGL((k_zfwd<T, SRC_MS_M>), dim3(a.g.tiles), dim3(a.g.nthr), lds_bytes, s, a); break;
    case SRC_RAW: hipLaunchKernelGGL((k_zfwd<T, SRC_RAW>), dim3(a.g.tiles), dim3(a.g.nthr), lds_bytes, s, a); break;
    default: hipLaunchKernelGGL((k_zfwd<T, SRC_ADJPRE>), dim3(a.g.tiles), dim3(a.g.nthr), lds_bytes, s, a); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_zinv(const ZInvArgs &a, int epi, size_t lds_bytes, hipStream_t s) {
    if (a.g.tiles <= 0) return hipSuccess;
    switch (epi) {
    case EPI_HEFF: hipLaunchKernelGGL((k_zinv<T, EPI_HEFF>), dim3(a.g.tiles), dim3(a.g.nthr), lds_bytes, s, a); break;
    case EPI_STAGE: hipLaunchKernelGGL((k_zinv<T, EPI_STAGE>), dim3(a.g.tiles), dim3(a.g.nthr), lds_bytes, s, a); break;
    case EPI_TAB: hipLaunchKernelGGL((k_zinv<T, EPI_TAB>), dim3(a.g.tiles), dim3(a.g.nthr), lds_bytes, s, a); break;
    case EPI_BB: hipLaunchKernelGGL((k_zinv<T, EPI_BB>), dim3(a.g.tiles), dim3(a.g.nthr), lds_bytes, s, a); break;
    default: hipLaunchKernelGGL((k_zinv<T, EPI_ADJ>), dim3(a.g.tiles), dim3(a.g.nthr), lds_bytes, s, a); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_zfwd_batch(const ZFwdArgs *d, const int2 *map, int tiles, int nthr, int src_mode, size_t lds_bytes,
                             hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    switch (src_mode) {
    case SRC_MS_M: hipLaunchKernelGGL((k_zfwd_b<T, SRC_MS_M>), dim3(tiles), dim3(nthr), lds_bytes, s, d, map); break;
    case SRC_RAW: hipLaunchKernelGGL((k_zfwd_b<T, SRC_RAW>), dim3(tiles), dim3(nthr), lds_bytes, s, d, map); break;
    default: hipLaunchKernelGGL((k_zfwd_b<T, SRC_ADJPRE>), dim3(tiles), dim3(nthr), lds_bytes, s, d, map); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_zinv_batch(const ZInvArgs *d, const int2 *map, int tiles, int nthr, int epi, size_t lds_bytes,
                             hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    switch (epi) {
    case EPI_HEFF: hipLaunchKernelGGL((k_zinv_b<T, EPI_HEFF>), dim3(tiles), dim3(nthr), lds_bytes, s, d, map); break;
    case EPI_STAGE: hipLaunchKernelGGL((k_zinv_b<T, EPI_STAGE>), dim3(tiles), dim3(nthr), lds_bytes, s, d, map); break;
    default: hipLaunchKernelGGL((k_zinv_b<T, EPI_ADJ>), dim3(tiles), dim3(nthr), lds_bytes, s, d, map); break;
    }
    return hipGetLastError();
}

template hipError_t launch_zfwd_batch<float>(const ZFwdArgs *, const int2 *, int, int, int, size_t, hipStream_t);
template hipError_t launch_zfwd_batch<double>(const ZFwdArgs *, const int2 *, int, int, int, size_t, hipStream_t);
template hipError_t launch_zinv_batch<float>(const ZInvArgs *, const int2 *, int, int, int, size_t, hipStream_t);
template hipError_t launch_zinv_batch<double>(const ZInvArgs *, const int2 *, int, int, int, size_t, hipStream_t);

// maximum of the per-block maxima (first of each pair), NaN propagating
__global__ void __launch_bounds__(256) k_max_reduce(const double *__restrict__ part, int nblk, double *out) {
    __shared__ double red[4];
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) v = nmax(v, part[2 * (int64_t)b]);
    block_max(v, red, out, threadIdx.x);
}

hipError_t launch_max_reduce(const double *part, int nblk, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, part, nblk, out);
    return hipGetLastError();
}

// minimiser: fixed-order sums of the per-block (s.s, s.y, y.y) and the
// maximum torque (one block of 256 threads)
__global__ void __launch_bounds__(256) k_bb_reduce(const double *__restrict__ part, int nblk, double *out4) {
    __shared__ double red[16];
    Acc4 acc;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        acc.v[0] += part[4 * (int64_t)b];
        acc.v[1] += part[4 * (int64_t)b + 1];
        acc.v[2] += part[4 * (int64_t)b + 2];
        acc.v[3] = nmax(acc.v[3], part[4 * (int64_t)b + 3]);
    }
    block_bb(acc, red, out4, threadIdx.x);
}

hipError_t launch_bb_reduce(const double *part, int nblk, double *out4, hipStream_t s) {
    hipLaunchKernelGGL(k_bb_reduce, dim3(1), dim3(256), 0, s, part, nblk, out4);
    return hipGetLastError();
}

// minimiser update: m_prev <- m, m <- (m - tau g) / |m - tau g| per cell
template <typename T>
__global__ void __launch_bounds__(256) k_bb_update(T *__restrict__ m, const T *__restrict__ g, T *__restrict__ mprev,
                                                   double tau, int64_t ncell) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncell) return;
    T u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T v = m[3 * i + c];
        mprev[3 * i + c] = v;
        u[c] = v - T(tau) * g[3 * i + c];
    }
    const T r = rnorm(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) m[3 * i + c] = u[c] * r;
}

template <typename T>
hipError_t launch_bb_update(T *m, const T *g, T *mprev, double tau, int64_t ncell, hipStream_t s) {
    if (ncell <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_bb_update<T>), dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, m, g, mprev, tau, ncell);
    return hipGetLastError();
}
template hipError_t launch_bb_update<float>(float *, const float *, float *, double, int64_t, hipStream_t);
template hipError_t launch_bb_update<double>(double *, const double *, double *, double, int64_t, hipStream_t);

hipError_t launch_energy_reduce(const double *part, int nblk, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_reduce, dim3(1), dim3(256), 0, s, part, nblk, out);
    return hipGetLastError();
}

template hipError_t launch_zfwd<float>(const ZFwdArgs &, int, size_t, hipStream_t);
template hipError_t launch_zfwd<double>(const ZFwdArgs &, int, size_t, hipStream_t);
template hipError_t launch_zinv<float>(const ZInvArgs &, int, size_t, hipStream_t);
template hipError_t launch_zinv<double>(const ZInvArgs &, int, size_t, hipStream_t);

}  // namespace mmx
