// Strided line passes (the y-axis passes of the convolution and the three
// real symmetric transforms of the tensor setup) and the fused x pass
// (forward FFT, spectral 3x3 product with the demag tensor, inverse FFT).
#include "passes.hpp"
#include "kernels.hpp"

namespace mmx {

// parity of component q (xx,yy,zz,xy,xz,yz) along axis a
__constant__ int kOdd[3][6] = {{0, 0, 0, 1, 1, 0}, {0, 0, 0, 1, 0, 1}, {0, 0, 0, 0, 1, 1}};

template <typename T, int DIR, bool SYM>
__global__ void __launch_bounds__(1024) k_line_pass(const LinePass *__restrict__ descs, const int2 *__restrict__ map) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const uint32_t t = xcd_tile(blockIdx.x, gridDim.x);
    int gi = 0, tile = (int)t;
    if (map) { const int2 e = map[t]; gi = e.x; tile = e.y; }
    const LinePass &a = descs[gi];
    const int tid = threadIdx.x, nthr = a.nthr;
    const int o = tile / a.tiles_inner;
    const int c0 = (tile - o * a.tiles_inner) * a.W;
    const int wc = min(a.W, a.inner - c0);
    const int L = a.f.L, pitch = a.pitch, n_in = a.n_in;
    if (tid < nthr) {
        if (!SYM) {
            const C *in = reinterpret_cast<const C *>(a.in) + (int64_t)o * a.in_outer + c0;
            for (int e = tid; e < n_in * wc; e += nthr) {
                const int r = e / wc, c = e - r * wc;
                lds[c * pitch + r] = in[(int64_t)r * a.in_row + c];
            }
            const C z = cmake<C>(T(0), T(0));
            for (int e = tid; e < (L - n_in) * wc; e += nthr) {
                const int r = n_in + e / wc, c = e % wc;
                lds[c * pitch + r] = z;
            }
        } else {
            // real line f(0..n-1) -> symmetric (even/odd) periodic extension
            const T *in = reinterpret_cast<const T *>(a.in) + (int64_t)o * a.in_outer + c0;
            for (int e = tid; e < n_in * wc; e += nthr) {
                const int r = e / wc, c = e - r * wc;
                const T v = in[(int64_t)r * a.in_row + c];
                const int odd = kOdd[a.sym_axis][(c0 + c) % 6];
                lds[c * pitch + r] = cmake<C>(v, T(0));
                if (r > 0) lds[c * pitch + (L - r)] = cmake<C>(odd ? -v : v, T(0));
            }
            const int nz = L - 2 * n_in + 1;   // slots n_in .. L-n_in are zero
            const C z = cmake<C>(T(0), T(0));
            for (int e = tid; e < nz * wc; e += nthr) {
                const int r = n_in + e / wc, c = e % wc;
                lds[c * pitch + r] = z;
            }
        }
    }
    __syncthreads();
    lds_fft<T, DIR>(lds, wc, pitch, a.f, reinterpret_cast<const C *>(a.tw), tid < nthr ? tid : 1 << 30, nthr);
    if (tid < nthr) {
        if (!SYM) {
            C *out = reinterpret_cast<C *>(a.out) + (int64_t)o * a.out_outer + c0;
            for (int e = tid; e < a.n_out * wc; e += nthr) {
                const int r = e / wc, c = e - r * wc;
                out[(int64_t)r * a.out_row + c] = lds[c * pitch + r];
            }
        } else {
            T *out = reinterpret_cast<T *>(a.out) + (int64_t)o * a.out_outer + c0;
            for (int e = tid; e < a.n_out * wc; e += nthr) {
                const int r = e / wc, c = e - r * wc;
                const C v = lds[c * pitch + r];
                const int odd = kOdd[a.sym_axis][(c0 + c) % 6];
                out[(int64_t)r * a.out_row + c] = odd ? -v.y : v.x;
            }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(1024) k_fused_x(const FusedPass *__restrict__ descs, const int2 *__restrict__ map) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const uint32_t t = xcd_tile(blockIdx.x, gridDim.x);
    int gi = 0, tile = (int)t;
    if (map) { const int2 e = map[t]; gi = e.x; tile = e.y; }
    const FusedPass &a = descs[gi];
    const int tid = threadIdx.x, nthr = a.nthr;
    const int p0 = tile * a.W;
    const int wp = min(a.W, a.npos - p0);
    const int nl = 3 * wp;
    const int L = a.f.L, pitch = a.pitch, n = a.n;
    C *data = reinterpret_cast<C *>(a.data) + (int64_t)p0 * 3;
    const C *tw = reinterpret_cast<const C *>(a.tw);
    const int ltid = tid < nthr ? tid : 1 << 30;
    if (tid < nthr) {
        for (int e = tid; e < n * nl; e += nthr) {
            const int r = e / nl, c = e - r * nl;
            lds[c * pitch + r] = data[(int64_t)r * a.row + c];
        }
        const C z = cmake<C>(T(0), T(0));
        for (int e = tid; e < (L - n) * nl; e += nthr) {
            const int r = n + e / nl, c = e % nl;
            lds[c * pitch + r] = z;
        }
    }
    __syncthreads();
    lds_fft<T, -1>(lds, nl, pitch, a.f, tw, ltid, nthr);
    if (tid < nthr) {
        const T *Nt = reinterpret_cast<const T *>(a.tensor);
        const int halfL = L / 2, halfY = a.Ly / 2;
        for (int e = tid; e < wp * L; e += nthr) {
            const int pl = e / L, kx = e - pl * L;
            const int p = p0 + pl;
            const int ky = p / a.hz, kz = p - ky * a.hz;
            const bool ry = ky > halfY, rx = kx > halfL;
            const int kyp = ry ? a.Ly - ky : ky, kxp = rx ? L - kx : kx;
            const T *N = Nt + ((int64_t)(kyp * a.hz + kz) * a.hx + kxp) * 6;
            const T sx = rx ? T(-1) : T(1), sy = ry ? T(-1) : T(1);
            const T nxx = N[0], nyy = N[1], nzz = N[2], nxy = N[3] * sx * sy, nxz = N[4] * sx, nyz = N[5] * sy;
            C *b = lds + (pl * 3) * pitch + kx;
            const C mx = b[0], my = b[pitch], mz = b[2 * pitch];
            b[0] = cmake<C>(nxx * mx.x + nxy * my.x + nxz * mz.x, nxx * mx.y + nxy * my.y + nxz * mz.y);
            b[pitch] = cmake<C>(nxy * mx.x + nyy * my.x + nyz * mz.x, nxy * mx.y + nyy * my.y + nyz * mz.y);
            b[2 * pitch] = cmake<C>(nxz * mx.x + nyz * my.x + nzz * mz.x, nxz * mx.y + nyz * my.y + nzz * mz.y);
        }
    }
    __syncthreads();
    lds_fft<T, +1>(lds, nl, pitch, a.f, tw, ltid, nthr);
    if (tid < nthr) {
        for (int e = tid; e < n * nl; e += nthr) {
            const int r = e / nl, c = e - r * nl;
            data[(int64_t)r * a.row + c] = lds[c * pitch + r];
        }
    }
}

template <typename T>
hipError_t launch_line_pass(const LinePass *d_descs, const int2 *d_map, int tiles, int nthr, size_t lds_bytes,
                            int dir, bool sym, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    if (sym) {
        if (dir < 0) hipLaunchKernelGGL((k_line_pass<T, -1, true>), dim3(tiles), dim3(nthr), lds_bytes, s, d_descs, d_map);
        else hipLaunchKernelGGL((k_line_pass<T, +1, true>), dim3(tiles), dim3(nthr), lds_bytes, s, d_descs, d_map);
    } else {
        if (dir < 0) hipLaunchKernelGGL((k_line_pass<T, -1, false>), dim3(tiles), dim3(nthr), lds_bytes, s, d_descs, d_map);
        else hipLaunchKernelGGL((k_line_pass<T, +1, false>), dim3(tiles), dim3(nthr), lds_bytes, s, d_descs, d_map);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fused_x(const FusedPass *d_descs, const int2 *d_map, int tiles, int nthr, size_t lds_bytes,
                          hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fused_x<T>), dim3(tiles), dim3(nthr), lds_bytes, s, d_descs, d_map);
    return hipGetLastError();
}

template hipError_t launch_line_pass<float>(const LinePass *, const int2 *, int, int, size_t, int, bool, hipStream_t);
template hipError_t launch_line_pass<double>(const LinePass *, const int2 *, int, int, size_t, int, bool, hipStream_t);
template hipError_t launch_fused_x<float>(const FusedPass *, const int2 *, int, int, size_t, hipStream_t);
template hipError_t launch_fused_x<double>(const FusedPass *, const int2 *, int, int, size_t, hipStream_t);

}  // namespace mmx
