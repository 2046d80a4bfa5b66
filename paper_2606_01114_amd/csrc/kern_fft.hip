// Strided line passes (the x-axis passes of the convolution and the three
// real symmetric transforms of the tensor setup) and the fused y pass
// (forward FFT, spectral 3x3 product with the demag tensor, inverse FFT) on
// contiguous three-component pencils.  Each comes as a runtime-planned kernel
// (any 7-smooth length, also used by grouped launches over many geometries)
// and as compile-time specialisations for power-of-two lengths.
#include "passes.hpp"
#include "kernels.hpp"
#include "fft_engine.hpp"
#include <algorithm>

namespace mmx {

// parity of component q (xx,yy,zz,xy,xz,yz) along axis a
__constant__ int kOdd[3][6] = {{0, 0, 0, 1, 1, 0}, {0, 0, 0, 1, 0, 1}, {0, 0, 0, 0, 1, 1}};

// ---------------- strided line pass --------------------------------------
template <typename T, bool SYM>
__device__ __forceinline__ void line_load(cplx<T> *lds, const LinePass &a, int o, int c0, int wc, int tid, int nthr) {
    using C = cplx<T>;
    const int L = a.f.L, pitch = a.pitch, n_in = a.n_in;
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

template <typename T, bool SYM>
__device__ __forceinline__ void line_store(const cplx<T> *lds, const LinePass &a, int o, int c0, int wc, int tid, int nthr) {
    using C = cplx<T>;
    const int pitch = a.pitch;
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
    if (tid < nthr) line_load<T, SYM>(lds, a, o, c0, wc, tid, nthr);
    __syncthreads();
    lds_fft<T, DIR>(lds, wc, a.pitch, a.f, reinterpret_cast<const C *>(a.tw), tid < nthr ? tid : 1 << 30, nthr);
    if (tid < nthr) line_store<T, SYM>(lds, a, o, c0, wc, tid, nthr);
}

// compile-time length L (power of two), W columns per tile, NT threads; the
// first stage loads from global memory, the last stores to global memory
template <typename T, int L, int DIR, int NT, int W>
__device__ __forceinline__ void line_ct_body(const LinePass &a, int tile) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const int o = tile / a.tiles_inner;
    const int c0 = (tile - o * a.tiles_inner) * W;
    const int wc = min(W, a.inner - c0);
    const int n_in = a.n_in, n_out = a.n_out;
    const uint32_t ir = (uint32_t)a.in_row * sizeof(C), orow = (uint32_t)a.out_row * sizeof(C);
    const C *in = reinterpret_cast<const C *>(a.in) + (int64_t)o * a.in_outer + c0;
    C *out = reinterpret_cast<C *>(a.out) + (int64_t)o * a.out_outer + c0;
    // each resource ends at the tile's last valid element: rows past n_in read
    // as zero, rows past n_out are not written
    const BufRsrc ri = make_rsrc(in, (uint32_t)(n_in - 1) * ir + (uint32_t)(a.inner - c0) * sizeof(C));
    const BufRsrc ro = make_rsrc(out, (uint32_t)(n_out - 1) * orow + (uint32_t)(a.inner - c0) * sizeof(C));
    // columns past the tile's width (last tile of a row) are loaded from the
    // next row or as zero and never stored
    auto ld = [&](int line, int pos) -> C { return buf_load<C>(ri, (uint32_t)pos * ir + (uint32_t)line * sizeof(C)); };
    auto st = [&](int line, int pos, C v) {
        buf_store(ro, (uint32_t)pos * orow + (line < wc ? (uint32_t)line * sizeof(C) : kBufOff), v);
    };
    // forward: input rows n_in <= L/2; inverse: output rows n_out <= L/2
    eng_fft<T, L, false, DIR, NT, W, DIR < 0 ? 1 : 2>(lds, reinterpret_cast<const C *>(a.tw), (int)threadIdx.x, ld, st);
}

template <typename T, int L, int DIR, int NT, int W>
__global__ void __launch_bounds__(NT) k_line_ct(const LinePass a) {
    line_ct_body<T, L, DIR, NT, W>(a, (int)xcd_tile(blockIdx.x, gridDim.x));
}

// grouped launch over many geometries of the same length L
template <typename T, int L, int DIR, int NT, int W>
__global__ void __launch_bounds__(NT) k_line_ct_b(const LinePass *__restrict__ descs, const int2 *__restrict__ map) {
    const int2 e = map[xcd_tile(blockIdx.x, gridDim.x)];
    line_ct_body<T, L, DIR, NT, W>(descs[e.x], e.y);
}

// x pass with register-resident lines and half-line LDS exchanges: the same
// tiles as k_line_ct at half the LDS, so two workgroups share a CU and one's
// global loads and stores overlap the other's exchanges and arithmetic.
template <typename T, int L, int DIR, int NT, int W>
__device__ __forceinline__ void line_hx_body(const LinePass &a, int tile) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const int o = tile / a.tiles_inner;
    const int c0 = (tile - o * a.tiles_inner) * W;
    const int wc = min(W, a.inner - c0);
    const uint32_t ir = (uint32_t)a.in_row * sizeof(C), orow = (uint32_t)a.out_row * sizeof(C);
    const C *in = reinterpret_cast<const C *>(a.in) + (int64_t)o * a.in_outer + c0;
    C *out = reinterpret_cast<C *>(a.out) + (int64_t)o * a.out_outer + c0;
    const BufRsrc ri = make_rsrc(in, (uint32_t)(a.n_in - 1) * ir + (uint32_t)(a.inner - c0) * sizeof(C));
    const BufRsrc ro = make_rsrc(out, (uint32_t)(a.n_out - 1) * orow + (uint32_t)(a.inner - c0) * sizeof(C));
    auto ld = [&](int line, int pos) -> C { return buf_load<C>(ri, (uint32_t)pos * ir + (uint32_t)line * sizeof(C)); };
    auto st = [&](int line, int pos, C v) {
        buf_store(ro, (uint32_t)pos * orow + (line < wc ? (uint32_t)line * sizeof(C) : kBufOff), v);
    };
    eng_fft_hx<T, L, DIR, NT, W, DIR < 0 ? 1 : 2>(lds, reinterpret_cast<const C *>(a.tw), (int)threadIdx.x, ld, st);
}

template <typename T, int L, int DIR, int NT, int W>
__global__ void __launch_bounds__(NT) k_line_hx(const LinePass a) {
    line_hx_body<T, L, DIR, NT, W>(a, (int)xcd_tile(blockIdx.x, gridDim.x));
}

// grouped launch over many geometries of the same length L
template <typename T, int L, int DIR, int NT, int W>
__global__ void __launch_bounds__(NT) k_line_hx_b(const LinePass *__restrict__ descs, const int2 *__restrict__ map) {
    const int2 e = map[xcd_tile(blockIdx.x, gridDim.x)];
    line_hx_body<T, L, DIR, NT, W>(descs[e.x], e.y);
}

// ---------------- fused y pass -------------------------------------------
// Pencil order within a kz plane pairs kx with Lx-kx (they read the same
// tensor row) so the two run close together: 0, [Lx/2], 1, Lx-1, 2, Lx-2, ...
__device__ __forceinline__ int pair_kx(int t, int Lx) {
    if (t == 0) return 0;
    if ((Lx & 1) == 0) {
        if (t == 1) return Lx / 2;
        const int u = (t - 2) / 2 + 1;
        return (t & 1) ? Lx - u : u;
    }
    const int u = (t - 1) / 2 + 1;
    return (t & 1) ? u : Lx - u;
}

// spectral product for the lines of one pencil held in LDS (3 lines, pitch)
template <typename T>
__device__ __forceinline__ void spectral_product(cplx<T> *b, int pitch, int ky, int Ly, const T *__restrict__ Trow,
                                                 T sx) {
    using C = cplx<T>;
    const bool ry = ky > Ly / 2;
    const int kyp = ry ? Ly - ky : ky;
    const T *N = Trow + (int64_t)kyp * 6;
    const T sy = ry ? T(-1) : T(1);
    const T nxx = N[0], nyy = N[1], nzz = N[2], nxy = N[3] * sx * sy, nxz = N[4] * sx, nyz = N[5] * sy;
    const C mx = b[ky], my = b[pitch + ky], mz = b[2 * pitch + ky];
    b[ky] = cmake<C>(nxx * mx.x + nxy * my.x + nxz * mz.x, nxx * mx.y + nxy * my.y + nxz * mz.y);
    b[pitch + ky] = cmake<C>(nxy * mx.x + nyy * my.x + nyz * mz.x, nxy * mx.y + nyy * my.y + nyz * mz.y);
    b[2 * pitch + ky] = cmake<C>(nxz * mx.x + nyz * my.x + nzz * mz.x, nxz * mx.y + nyz * my.y + nzz * mz.y);
}

template <typename T>
__global__ void __launch_bounds__(1024) k_fused_y(const FusedPass *__restrict__ descs, const int2 *__restrict__ map) {
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
    const int L = a.f.L, pitch = a.pitch, n = a.n, n3 = 3 * n;
    const C *tw = reinterpret_cast<const C *>(a.tw);
    const int ltid = tid < nthr ? tid : 1 << 30;
    C *data = reinterpret_cast<C *>(a.data);
    if (tid < nthr) {
        for (int pl = 0; pl < wp; ++pl) {
            const int p = p0 + pl, kz = p / a.Lx, kx = pair_kx(p - kz * a.Lx, a.Lx);
            const C *src = data + ((int64_t)kz * a.Lx + kx) * n3;
            C *b = lds + pl * 3 * pitch;
            for (int e = tid; e < n3; e += nthr) {
                const int j = e / 3, c = e - 3 * j;
                b[c * pitch + j] = src[e];
            }
            const C z = cmake<C>(T(0), T(0));
            for (int e = tid; e < 3 * (L - n); e += nthr) {
                const int c = e / (L - n), j = n + (e - c * (L - n));
                b[c * pitch + j] = z;
            }
        }
    }
    __syncthreads();
    lds_fft<T, -1>(lds, 3 * wp, pitch, a.f, tw, ltid, nthr);
    if (tid < nthr) {
        const T *Nt = reinterpret_cast<const T *>(a.tensor);
        for (int e = tid; e < wp * L; e += nthr) {
            const int pl = e / L, ky = e - pl * L;
            const int p = p0 + pl, kz = p / a.Lx, kx = pair_kx(p - kz * a.Lx, a.Lx);
            const bool rx = kx > a.Lx / 2;
            const int kxp = rx ? a.Lx - kx : kx;
            spectral_product<T>(lds + pl * 3 * pitch, pitch, ky, L, Nt + ((int64_t)kz * a.hxp + kxp) * a.hyp * 6,
                                rx ? T(-1) : T(1));
        }
    }
    __syncthreads();
    lds_fft<T, +1>(lds, 3 * wp, pitch, a.f, tw, ltid, nthr);
    if (tid < nthr) {
        for (int pl = 0; pl < wp; ++pl) {
            const int p = p0 + pl, kz = p / a.Lx, kx = pair_kx(p - kz * a.Lx, a.Lx);
            C *dst = data + ((int64_t)kz * a.Lx + kx) * n3;
            const C *b = lds + pl * 3 * pitch;
            for (int e = tid; e < n3; e += nthr) {
                const int j = e / 3, c = e - 3 * j;
                dst[e] = b[c * pitch + j];
            }
        }
    }
}

// The middle of the convolution of one three-line pencil held in LDS: the
// last forward radix stage, the 3x3 spectral product and the first inverse
// stage, all in registers (the inverse runs its radices in reversed order, so
// its first stage reads exactly the positions the last forward stage
// produced).  Reads and writes LDS; ends with a barrier.
template <typename T, int L, int NT, class Pr, int TM = 0>
__device__ __forceinline__ void conv_middle(cplx<T> *lds, const cplx<T> *__restrict__ twf, int tid, const Pr &prod) {
    using C = cplx<T>;
    constexpr int NS = ct::nst(L);
    constexpr int P = ct::lds_pitch(L, 3, (int)sizeof(cplx<T>));
    constexpr int R = ct::prad(L, false, NS - 1);
    constexpr int NB = L / R;
    constexpr int Nsf = ct::pns(L, false, NS - 1);
    constexpr int TWM = ct::ptw(L, false, NS - 1);
    constexpr int UJ = (NB + NT - 1) / NT;
    C v[UJ][3][R];
#pragma unroll
    for (int u = 0; u < UJ; ++u) {
        const int j = tid + u * NT;
        if (j < NB) {
            const int sj = sw<L>(j);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[u][c][r] = lds[c * P + sj + swc<L>(r * NB)];
                if (Nsf > 1) {
                    const int k = j % Nsf;
                    const C *tt = twf + TWM + k * (R - 1);
#pragma unroll
                    for (int r = 1; r < R; ++r) v[u][c][r] = cmul(v[u][c][r], stage_tw<L, Nsf, R, TM>(twf, tt, k, r));
                }
                Dft<R, -1, C>::run(v[u][c]);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) prod(j + r * NB, v[u][0][r], v[u][1][r], v[u][2][r]);
#pragma unroll
            for (int c = 0; c < 3; ++c) Dft<R, +1, C>::run(v[u][c]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UJ; ++u) {
        const int j = tid + u * NT;
        if (j < NB) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int r = 0; r < R; ++r) lds[c * P + swb<L, R>(j * R, r)] = v[u][c][r];
        }
    }
    __syncthreads();
}

// Tensor values a thread of conv_middle needs, fetched before the transform
// starts so their latency overlaps the first radix stages: tv[u][r][q] for
// ky = j + r NB, j = tid + u NT, with the odd components' sign flips applied.
template <typename T, int L, int NT>
struct PencilTensor {
    static constexpr int NS = ct::nst(L);
    static constexpr int R = ct::prad(L, false, NS - 1);
    static constexpr int NB = L / R;
    static constexpr int UJ = (NB + NT - 1) / NT;
    T tv[UJ][R][6];
    __device__ __forceinline__ void load(const T *__restrict__ Trow, T sx, int tid) {
#pragma unroll
        for (int u = 0; u < UJ; ++u) {
            const int j = tid + u * NT;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int ky = j + r * NB;
                const bool ry = ky > L / 2;
                const int kyp = ry ? L - ky : ky;
                const T sy = ry ? T(-1) : T(1);
                if (j < NB) {
                    const T *N = Trow + kyp * 6;
#pragma unroll
                    for (int q = 0; q < 6; ++q) tv[u][r][q] = N[q];
                    tv[u][r][3] *= sx * sy;
                    tv[u][r][4] *= sx;
                    tv[u][r][5] *= sy;
                }
            }
        }
    }
};

// conv_middle with the tensor already in registers (TM: twiddle table form,
// as for eng_stage_la)
template <typename T, int L, int NT, int TM = 0>
__device__ __forceinline__ void conv_middle_pre(cplx<T> *lds, const cplx<T> *__restrict__ twf, int tid,
                                                const PencilTensor<T, L, NT> &pt) {
    using C = cplx<T>;
    constexpr int NS = ct::nst(L);
    constexpr int P = ct::lds_pitch(L, 3, (int)sizeof(cplx<T>));
    constexpr int R = ct::prad(L, false, NS - 1);
    constexpr int NB = L / R;
    constexpr int Nsf = ct::pns(L, false, NS - 1);
    constexpr int TWM = ct::ptw(L, false, NS - 1);
    constexpr int UJ = (NB + NT - 1) / NT;
    C v[UJ][3][R];
#pragma unroll
    for (int u = 0; u < UJ; ++u) {
        const int j = tid + u * NT;
        if (j < NB) {
            const int sj = sw<L>(j);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[u][c][r] = lds[c * P + sj + swc<L>(r * NB)];
                if (Nsf > 1) {
                    const int k = j % Nsf;
                    const C *tt = twf + TWM + k * (R - 1);
#pragma unroll
                    for (int r = 1; r < R; ++r) v[u][c][r] = cmul(v[u][c][r], stage_tw<L, Nsf, R, TM>(twf, tt, k, r));
                }
                Dft<R, -1, C>::run(v[u][c]);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T *N = pt.tv[u][r];
                const C x = v[u][0][r], y = v[u][1][r], z = v[u][2][r];
                v[u][0][r] = cmake<C>(N[0] * x.x + N[3] * y.x + N[4] * z.x, N[0] * x.y + N[3] * y.y + N[4] * z.y);
                v[u][1][r] = cmake<C>(N[3] * x.x + N[1] * y.x + N[5] * z.x, N[3] * x.y + N[1] * y.y + N[5] * z.y);
                v[u][2][r] = cmake<C>(N[4] * x.x + N[5] * y.x + N[2] * z.x, N[4] * x.y + N[5] * y.y + N[2] * z.y);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) Dft<R, +1, C>::run(v[u][c]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UJ; ++u) {
        const int j = tid + u * NT;
        if (j < NB) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int r = 0; r < R; ++r) lds[c * P + swb<L, R>(j * R, r)] = v[u][c][r];
        }
    }
    __syncthreads();
}

// tensor product of one (kz, kx) pencil: the tensor row (kz, |kx|) with the
// sign flips of the odd components under kx -> Lx-kx and ky -> Ly-ky
template <typename T, int L>
struct PencilProduct {
    const T *Trow;
    T sx;
    __device__ __forceinline__ void operator()(int ky, cplx<T> &mx, cplx<T> &my, cplx<T> &mz) const {
        using C = cplx<T>;
        const bool ry = ky > L / 2;
        const int kyp = ry ? L - ky : ky;
        const T *N = Trow + kyp * 6;
        const T sy = ry ? T(-1) : T(1);
        const T nxx = N[0], nyy = N[1], nzz = N[2], nxy = N[3] * sx * sy, nxz = N[4] * sx, nyz = N[5] * sy;
        const C x = mx, y = my, z = mz;
        mx = cmake<C>(nxx * x.x + nxy * y.x + nxz * z.x, nxx * x.y + nxy * y.y + nxz * z.y);
        my = cmake<C>(nxy * x.x + nyy * y.x + nyz * z.x, nxy * x.y + nyy * y.y + nyz * z.y);
        mz = cmake<C>(nxz * x.x + nyz * y.x + nzz * z.x, nxz * x.y + nyz * y.y + nzz * z.y);
    }
};

template <typename T, int L>
__device__ __forceinline__ PencilProduct<T, L> pencil_product(const FusedPass &a, int kz, int kx) {
    const bool rx = kx > a.Lx / 2;
    const int kxp = rx ? a.Lx - kx : kx;
    PencilProduct<T, L> pr;
    pr.Trow = reinterpret_cast<const T *>(a.tensor) + ((int64_t)kz * a.hxp + kxp) * a.hyp * 6;
    pr.sx = rx ? T(-1) : T(1);
    return pr;
}

// compile-time Ly; one (kz, kx) pencil of three components per tile.  The
// tensor row is fetched into registers together with the pencil's first
// radix-stage inputs.
// rot: the workgroup's waves take the butterflies of the wave rot places on,
// so that when a stage has fewer butterflies than threads in its last round
// the busy waves differ from workgroup to workgroup and the SIMDs of a CU
// share the uneven rounds.
template <typename T, int L, int NT>
__device__ __forceinline__ void fused_ct_body(const FusedPass &a, int p, int rot = 0) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    constexpr int NS = ct::nst(L);
    static_assert(NS >= 2, "fused pencil needs two or more radix stages");
    const int tid = (NT & (NT - 1)) == 0 ? (int)(threadIdx.x ^ (64u * (unsigned)rot))
                                         : (int)((threadIdx.x + 64u * (unsigned)rot) % (unsigned)NT);
    const int n = a.n;
    const int kz = p / a.Lx, kx = pair_kx(p - kz * a.Lx, a.Lx);
    C *pen = reinterpret_cast<C *>(a.data) + ((int64_t)kz * a.Lx + kx) * (3 * n);
    const bool rx = kx > a.Lx / 2;
    const int kxp = rx ? a.Lx - kx : kx;
    const T *Trow = reinterpret_cast<const T *>(a.tensor) + ((int64_t)kz * a.hxp + kxp) * a.hyp * 6;
    const T sx = rx ? T(-1) : T(1);
    // FP32: fetch the tensor early (registers to spare); FP64: at the product
    constexpr bool early = sizeof(T) == 4;
    PencilTensor<T, L, (early ? NT : 1)> pt;
    if constexpr (early) pt.load(Trow, sx, tid);
    // rows past n (the zero padding) read as zero and are not written
    const BufRsrc rp = make_rsrc(pen, (uint32_t)(3 * n) * sizeof(C));
    auto ld = [&](int c, int pos) -> C { return buf_load<C>(rp, (uint32_t)(pos * 3 + c) * sizeof(C)); };
    auto st = [&](int c, int pos, C v) { buf_store(rp, (uint32_t)(pos * 3 + c) * sizeof(C), v); };
    const C *tw = reinterpret_cast<const C *>(a.tw);
    const C *twr = tw + (L - 1);
    auto nost = [](int, int, C) {};
    auto nold = [](int, int) { return C(); };
    eng_stage<T, L, false, 0, -1, NT, 3, 0, 1, 1>(lds, tw, tid, ld, nost);
    eng_mid<T, L, false, 1, NS - 1, -1, NT, 3>(lds, tw, tid);
    if constexpr (early) {
        conv_middle_pre<T, L, NT>(lds, tw, tid, pt);
    } else {
        PencilProduct<T, L> pr;
        pr.Trow = Trow;
        pr.sx = sx;
        conv_middle<T, L, NT>(lds, tw, tid, pr);
    }
    eng_mid<T, L, true, 1, NS - 1, +1, NT, 3>(lds, twr, tid);
    eng_stage<T, L, true, NS - 1, +1, NT, 3, 1, 0, 2>(lds, twr, tid, nold, st);
}

// ---- fused y pass with register-resident pencils ---------------------------
// The pencil's values stay in registers from the first forward stage to the
// last inverse stage; the stages exchange them through an LDS buffer of half
// a line per component (lower half of the positions first, then the upper
// half), so a workgroup needs half the LDS of k_fused_y_ct and more pencils
// share a CU.  The middle (last forward stage, tensor product, first inverse
// stage) runs on triples: one thread holds all three components of its ky.
template <int L, int NT> struct FusedHx {
    static constexpr int NS = ct::nst(L);
    static constexpr int RC = ct::prad(L, false, NS - 1);
    static constexpr int NBC = L / RC;
    static constexpr int UC = (NBC + NT - 1) / NT;
    static constexpr int PH = hx_pitch<L, 3, 8>();   // the three-line shift is the same for both value sizes
};

// forward stage S's outputs v -> ... -> the middle's inputs vc
template <typename T, int L, int NT, int S, int U, int R>
__device__ __forceinline__ void fhx_forward(cplx<T> *lds, cplx<T> (&v)[U][R],
                                            cplx<T> (&vc)[FusedHx<L, NT>::UC][3][FusedHx<L, NT>::RC],
                                            const cplx<T> *__restrict__ tw, int tid) {
    using F = FusedHx<L, NT>;
    if constexpr (S + 1 == F::NS - 1) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            hx_put<T, L, false, S, NT, 3>(lds, v, h, tid);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < F::UC; ++u) {
                const int j = tid + u * NT;
                if (j < F::NBC) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const int base = c * F::PH + sw<L>(j);
#pragma unroll
                        for (int r = 0; r < F::RC / 2; ++r) vc[u][c][h * (F::RC / 2) + r] = lds[base + swc<L>(r * F::NBC)];
                    }
                }
            }
            __syncthreads();
        }
    } else {
        using B = HxStage<L, false, S + 1>;
        constexpr int UI = (3 * B::NB + NT - 1) / NT;
        cplx<T> w[UI][B::R];
        hx_exchange<T, L, false, S, NT, 3>(lds, v, w, tid);
        hx_compute<T, L, false, S + 1, -1, NT, 3, 0>(w, tw, tid);
        fhx_forward<T, L, NT, S + 1>(lds, w, vc, tw, tid);
    }
}

// inverse stage S (reversed order) from its inputs v; the last stage stores
// the rows below L/2 (rows at or past n are dropped by the resource)
template <typename T, int L, int NT, int S, int U, int R>
__device__ __forceinline__ void fhx_inverse(cplx<T> *lds, cplx<T> (&v)[U][R], const cplx<T> *__restrict__ twr,
                                            int tid, BufRsrc rp) {
    using C = cplx<T>;
    constexpr int NS = ct::nst(L);
    constexpr bool LAST = S == NS - 1;
    hx_compute<T, L, true, S, +1, NT, 3, LAST ? 2 : 0>(v, twr, tid);
    if constexpr (LAST) {
        using A = HxStage<L, true, S>;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = tid + u * NT;
            if (b < 3 * A::NB) {
                const int line = b % 3, j = b / 3;
                const int d = (j / A::Ns) * A::Ns * R + (j % A::Ns);
#pragma unroll
                for (int r = 0; r < R / 2; ++r) buf_store(rp, (uint32_t)((d + r * A::Ns) * 3 + line) * sizeof(C), v[u][r]);
            }
        }
    } else {
        using B = HxStage<L, true, S + 1>;
        constexpr int UI = (3 * B::NB + NT - 1) / NT;
        C w[UI][B::R];
        hx_exchange<T, L, true, S, NT, 3>(lds, v, w, tid);
        fhx_inverse<T, L, NT, S + 1>(lds, w, twr, tid, rp);
    }
}

template <typename T, int L, int NT>
__device__ __forceinline__ void fused_hx_body(const FusedPass &a, int p) {
    using C = cplx<T>;
    using F = FusedHx<L, NT>;
    static_assert(F::NS >= 2, "fused pencil needs two or more radix stages");
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const int tid = threadIdx.x;
    const int n = a.n;
    const int kz = p / a.Lx, kx = pair_kx(p - kz * a.Lx, a.Lx);
    C *pen = reinterpret_cast<C *>(a.data) + ((int64_t)kz * a.Lx + kx) * (3 * n);
    const BufRsrc rp = make_rsrc(pen, (uint32_t)(3 * n) * sizeof(C));
    const PencilProduct<T, L> pr = pencil_product<T, L>(a, kz, kx);
    const C *tw = reinterpret_cast<const C *>(a.tw);
    const C *twr = tw + (L - 1);
    // forward stage 0 straight from the pencil (rows past L/2 are padding)
    using A0 = HxStage<L, false, 0>;
    constexpr int U0 = (3 * A0::NB + NT - 1) / NT;
    C v0[U0][A0::R];
#pragma unroll
    for (int u = 0; u < U0; ++u) {
        const int b = tid + u * NT;
        if (b < 3 * A0::NB) {
            const int line = b % 3, j = b / 3;
#pragma unroll
            for (int r = 0; r < A0::R / 2; ++r) v0[u][r] = buf_load<C>(rp, (uint32_t)((j + r * A0::NB) * 3 + line) * sizeof(C));
            PDft<A0::R, -1, 1, C>::run(v0[u]);
        }
    }
    C vc[F::UC][3][F::RC];
    fhx_forward<T, L, NT, 0>(lds, v0, vc, tw, tid);
    // middle: last forward stage, 3x3 product, first inverse stage
    constexpr int Nsf = ct::pns(L, false, F::NS - 1);
    constexpr int TWM = ct::ptw(L, false, F::NS - 1);
#pragma unroll
    for (int u = 0; u < F::UC; ++u) {
        const int j = tid + u * NT;
        if (j < F::NBC) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (Nsf > 1) {
                    const C *tt = tw + TWM + (j % Nsf) * (F::RC - 1);
#pragma unroll
                    for (int r = 1; r < F::RC; ++r) vc[u][c][r] = cmul(vc[u][c][r], tt[r - 1]);
                }
                Dft<F::RC, -1, C>::run(vc[u][c]);
            }
#pragma unroll
            for (int r = 0; r < F::RC; ++r) pr(j + r * F::NBC, vc[u][0][r], vc[u][1][r], vc[u][2][r]);
#pragma unroll
            for (int c = 0; c < 3; ++c) Dft<F::RC, +1, C>::run(vc[u][c]);
        }
    }
    // middle -> inverse stage 1 (outputs of the first inverse stage sit at
    // j RC + r: one block of RC per triple, in one half of the line)
    using B1 = HxStage<L, true, 1>;
    constexpr int U1 = (3 * B1::NB + NT - 1) / NT;
    C w1[U1][B1::R];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int u = 0; u < F::UC; ++u) {
            const int j = tid + u * NT;
            if (j < F::NBC && (j >= F::NBC / 2) == (h == 1)) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int base = c * F::PH + sw<L>(j * F::RC - h * (L / 2));
#pragma unroll
                    for (int r = 0; r < F::RC; ++r) lds[base + swc<L>(r)] = vc[u][c][r];
                }
            }
        }
        __syncthreads();
        hx_get<T, L, true, 1, NT, 3>(lds, w1, h, tid);
        __syncthreads();
    }
    fhx_inverse<T, L, NT, 1>(lds, w1, twr, tid, rp);
}

template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT) k_fused_y_hx(const FusedPass a) {
    fused_hx_body<T, L, NT>(a, (int)xcd_tile(blockIdx.x, gridDim.x));
}

template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT) k_fused_y_ct(const FusedPass a) {
    fused_ct_body<T, L, NT>(a, (int)xcd_tile(blockIdx.x, gridDim.x));
}

// k_fused_y_ct with the waves' butterflies rotated per workgroup
template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT) k_fused_y_cr(const FusedPass a) {
    fused_ct_body<T, L, NT>(a, (int)xcd_tile(blockIdx.x, gridDim.x), (int)((blockIdx.x >> 3) % (NT / 64)));
}

template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT) k_fused_y_ct_b(const FusedPass *__restrict__ descs, const int2 *__restrict__ map) {
    const int2 e = map[xcd_tile(blockIdx.x, gridDim.x)];
    fused_ct_body<T, L, NT>(descs[e.x], e.y);
}

// grouped launches of the wave-rotated and register-resident variants
template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT) k_fused_y_cr_b(const FusedPass *__restrict__ descs, const int2 *__restrict__ map) {
    const int2 e = map[xcd_tile(blockIdx.x, gridDim.x)];
    fused_ct_body<T, L, NT>(descs[e.x], e.y, (int)((blockIdx.x >> 3) % (NT / 64)));
}

template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT) k_fused_y_hx_b(const FusedPass *__restrict__ descs, const int2 *__restrict__ map) {
    const int2 e = map[xcd_tile(blockIdx.x, gridDim.x)];
    fused_hx_body<T, L, NT>(descs[e.x], e.y);
}

// ---- fused y pass, persistent, with the next pencil's loads in flight -----
// The first forward stage's inputs of one pencil (the rows below L/2 of its
// three components), held in registers between their load and the stage.
template <typename T, int L, int NT>
struct PencilInputs {
    using C = cplx<T>;
    static constexpr int R = ct::prad(L, false, 0);
    static constexpr int NB = L / R;
    static constexpr int TOT = 3 * NB;
    static constexpr int U = (TOT + NT - 1) / NT;
    C v[U][R / 2];
    // butterfly b = tid + u NT reads line b % 3 at rows j + r NB, j = b / 3
    __device__ __forceinline__ void load(BufRsrc rp, int tid) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = tid + u * NT;
            if (b < TOT) {
                const int line = b % 3, j = b / 3;
#pragma unroll
                for (int r = 0; r < R / 2; ++r) v[u][r] = buf_load<C>(rp, (uint32_t)((j + r * NB) * 3 + line) * sizeof(C));
            }
        }
    }
    // the first stage (no twiddles, upper half of every input zero) into LDS;
    // ends with a barrier
    __device__ __forceinline__ void stage0(C *lds, int tid) const {
        constexpr int P = ct::lds_pitch(L, 3, (int)sizeof(C));
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = tid + u * NT;
            if (b < TOT) {
                const int line = b % 3, j = b / 3;
                C w[R];
#pragma unroll
                for (int r = 0; r < R / 2; ++r) w[r] = v[u][r];
                PDft<R, -1, 1, C>::run(w);
                const int sd = line * P + sw<L>(j * R);
#pragma unroll
                for (int r = 0; r < R; ++r) lds[sd + swc<L>(r)] = w[r];
            }
        }
        __syncthreads();
    }
};

// Persistent form of fused_ct_body: a resident grid walks the pencils; the
// first stage's global loads of the workgroup's next pencil are issued as
// soon as the current pencil's first stage has consumed its own, so their
// latency overlaps the remaining stages instead of stalling every pencil's
// start.  Virtual tile v = blockIdx.x + i gridDim.x maps to a pencil through
// xcd_tile, so each XCD's workgroups (gridDim.x a multiple of 8) walk that
// XCD's contiguous run of pencils side by side.  EARLY: fetch the pencil's
// tensor values when the pencil starts (else at the product).
template <typename T, int L, int NT, bool EARLY, int MINW = 1>
__global__ void __launch_bounds__(NT, MINW) k_fused_y_pf(const FusedPass a) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    constexpr int NS = ct::nst(L);
    static_assert(NS >= 2, "fused pencil needs two or more radix stages");
    // waves rotated per workgroup as in k_fused_y_cr
    const unsigned rot = (blockIdx.x >> 3) % (NT / 64);
    const int tid = (NT & (NT - 1)) == 0 ? (int)(threadIdx.x ^ (64u * rot)) : (int)((threadIdx.x + 64u * rot) % (unsigned)NT);
    const int n = a.n, G = (int)gridDim.x, npos = a.npos;
    const C *tw = reinterpret_cast<const C *>(a.tw);
    const C *twr = tw + (L - 1);
    auto pencil = [&](int v) {
        const int p = (int)xcd_tile((uint32_t)v, (uint32_t)npos);
        const int kz = p / a.Lx;
        return make_int2(kz, pair_kx(p - kz * a.Lx, a.Lx));
    };
    auto rsrc = [&](int2 q) {
        C *pen = reinterpret_cast<C *>(a.data) + ((int64_t)q.x * a.Lx + q.y) * (3 * n);
        return make_rsrc(pen, (uint32_t)(3 * n) * sizeof(C));
    };
    int v = (int)blockIdx.x;
    if (v >= npos) return;
    PencilInputs<T, L, NT> in;
    int2 q = pencil(v);
    in.load(rsrc(q), tid);
    auto nold = [](int, int) { return C(); };
    for (; v < npos; v += G) {
        const BufRsrc rp = rsrc(q);
        auto st = [&](int c, int pos, C x) { buf_store(rp, (uint32_t)(pos * 3 + c) * sizeof(C), x); };
        const bool rx = q.y > a.Lx / 2;
        const T *Trow = reinterpret_cast<const T *>(a.tensor) + ((int64_t)q.x * a.hxp + (rx ? a.Lx - q.y : q.y)) * a.hyp * 6;
        const T sx = rx ? T(-1) : T(1);
        PencilTensor<T, L, (EARLY ? NT : 1)> pt;
        if constexpr (EARLY) pt.load(Trow, sx, tid);
        // the previous pencil's last stage has finished reading LDS
        __syncthreads();
        in.stage0(lds, tid);
        const int vn = v + G;
        const int2 qn = vn < npos ? pencil(vn) : q;
        if (vn < npos) in.load(rsrc(qn), tid);
        eng_mid<T, L, false, 1, NS - 1, -1, NT, 3>(lds, tw, tid);
        if constexpr (EARLY) {
            conv_middle_pre<T, L, NT>(lds, tw, tid, pt);
        } else {
            PencilProduct<T, L> pr;
            pr.Trow = Trow;
            pr.sx = sx;
            conv_middle<T, L, NT>(lds, tw, tid, pr);
        }
        eng_mid<T, L, true, 1, NS - 1, +1, NT, 3>(lds, twr, tid);
        eng_stage<T, L, true, NS - 1, +1, NT, 3, 1, 0, 2>(lds, twr, tid, nold, st);
        q = qn;
    }
}

// Persistent fused pass with the twiddles in LDS: the Ly roots
// exp(-2 pi i m / Ly) sit behind the pencil, copied once per workgroup, so no
// radix stage waits on a global twiddle load.  The only global loads are the
// next pencil's first-stage inputs, issued right after the first stage, and
// the current pencil's tensor values (EARLY: issued with them, so the forward
// stages cover their latency; else at the product, which saves registers).
// Waits on global loads complete in issue order, so a twiddle load between
// the prefetch and its use would wait for the prefetch too.
template <typename T, int L, int NT, bool EARLY>
__global__ void __launch_bounds__(NT) k_fused_y_pt(const FusedPass a) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    constexpr int NS = ct::nst(L);
    static_assert(NS >= 2, "fused pencil needs two or more radix stages");
    constexpr int P = ct::lds_pitch(L, 3, (int)sizeof(C));
    C *roots = lds + 3 * P;
    const unsigned rot = (blockIdx.x >> 3) % (NT / 64);
    const int tid = (NT & (NT - 1)) == 0 ? (int)(threadIdx.x ^ (64u * rot)) : (int)((threadIdx.x + 64u * rot) % (unsigned)NT);
    const int n = a.n, G = (int)gridDim.x, npos = a.npos;
    int v = (int)blockIdx.x;
    if (v >= npos) return;
    {
        const C *rg = reinterpret_cast<const C *>(a.roots);
        for (int i = (int)threadIdx.x; i < L; i += NT) roots[i] = rg[i];
    }
    auto pencil = [&](int vv) {
        const int p = (int)xcd_tile((uint32_t)vv, (uint32_t)npos);
        const int kz = p / a.Lx;
        return make_int2(kz, pair_kx(p - kz * a.Lx, a.Lx));
    };
    auto rsrc = [&](int2 qq) {
        C *pen = reinterpret_cast<C *>(a.data) + ((int64_t)qq.x * a.Lx + qq.y) * (3 * n);
        return make_rsrc(pen, (uint32_t)(3 * n) * sizeof(C));
    };
    PencilInputs<T, L, NT> in;
    int2 q = pencil(v);
    in.load(rsrc(q), tid);
    auto nold = [](int, int) { return C(); };
    for (; v < npos; v += G) {
        const BufRsrc rp = rsrc(q);
        auto st = [&](int c, int pos, C x) { buf_store(rp, (uint32_t)(pos * 3 + c) * sizeof(C), x); };
        const bool rx = q.y > a.Lx / 2;
        const T *Trow = reinterpret_cast<const T *>(a.tensor) + ((int64_t)q.x * a.hxp + (rx ? a.Lx - q.y : q.y)) * a.hyp * 6;
        const T sx = rx ? T(-1) : T(1);
        // the previous pencil's last stage has finished reading LDS (first
        // pencil: the roots are in place)
        __syncthreads();
        in.stage0(lds, tid);
        PencilTensor<T, L, (EARLY ? NT : 1)> pt;
        if constexpr (EARLY) pt.load(Trow, sx, tid);
        const int vn = v + G;
        const int2 qn = vn < npos ? pencil(vn) : q;
        if (vn < npos) in.load(rsrc(qn), tid);
        eng_mid<T, L, false, 1, NS - 1, -1, NT, 3, 1>(lds, roots, tid);
        if constexpr (EARLY) {
            conv_middle_pre<T, L, NT, 1>(lds, roots, tid, pt);
        } else {
            PencilProduct<T, L> pr;
            pr.Trow = Trow;
            pr.sx = sx;
            conv_middle<T, L, NT, PencilProduct<T, L>, 1>(lds, roots, tid, pr);
        }
        eng_mid<T, L, true, 1, NS - 1, +1, NT, 3, 1>(lds, roots, tid);
        eng_stage<T, L, true, NS - 1, +1, NT, 3, 1, 0, 2, 1>(lds, roots, tid, nold, st);
        q = qn;
    }
}

// ---- fused y pass in two half-spectra --------------------------------------
// The upper half of each y line is zero and only the lower half of the result
// is kept, so the Ly-point convolution splits exactly into two of Ly/2
// points: the even frequencies ky = 2m are the Ly/2-point DFT of x_n, the odd
// ones ky = 2m+1 the Ly/2-point DFT of w^n x_n (w = exp(-2 pi i / Ly)), and
// each kept output is the even half's Ly/2-point inverse plus w^-n times the
// odd half's.  A workgroup runs the two halves one after the other through an
// LDS pencil of Ly/2 positions (half the LDS of k_fused_y_ct, so that more
// pencils share a CU).  The first stage's inputs stay in registers for the
// odd half and the even half's outputs until the odd half's are added, so the
// pencil is read and written once.  Those reads and writes carry the
// streaming hint: the caches then keep the tensor row, which both halves read
// (and the neighbouring pencil, kx -> Lx - kx, after them).
template <typename T, int L, int H> struct HalfProduct {
    PencilProduct<T, L> pr;
    __device__ __forceinline__ void operator()(int m, cplx<T> &x, cplx<T> &y, cplx<T> &z) const { pr(2 * m + H, x, y, z); }
};

template <typename T, int L, int NT, int H, int U, int R, int UI, int RI>
__device__ __forceinline__ void h2_half(cplx<T> *lds, const FusedPass &a, const BufRsrc &rp, const PencilProduct<T, L> &pr,
                                        cplx<T> (&acc)[U][R], cplx<T> (&xin)[UI][RI], int tid) {
    using C = cplx<T>;
    constexpr int M = L / 2;
    constexpr int NS = ct::nst(M);
    const C *twh = reinterpret_cast<const C *>(a.twh);
    const C *twhr = twh + (M - 1);
    const C *roots = reinterpret_cast<const C *>(a.roots);
    auto ld = [&](int u, int r, int c, int pos) -> C {
        if constexpr (H == 0) {
            xin[u][r] = buf_load_nt<C>(rp, (uint32_t)(pos * 3 + c) * sizeof(C));
            return xin[u][r];
        } else {
            return cmul(xin[u][r], roots[pos]);
        }
    };
    auto nost = [](int, int, C) {};
    auto nold = [](int, int) { return C(); };
    eng_stage<T, M, false, 0, -1, NT, 3, 2, 1>(lds, twh, tid, ld, nost);
    eng_mid<T, M, false, 1, NS - 1, -1, NT, 3>(lds, twh, tid);
    HalfProduct<T, L, H> hp{pr};
    conv_middle<T, M, NT>(lds, twh, tid, hp);
    eng_mid<T, M, true, 1, NS - 1, +1, NT, 3>(lds, twhr, tid);
    auto st = [&](int u, int r, int c, int pos, C v) {
        if constexpr (H == 0) acc[u][r] = v;
        else buf_store_nt(rp, (uint32_t)(pos * 3 + c) * sizeof(C), cadd(acc[u][r], cmul(cconj(roots[pos]), v)));
    };
    eng_stage<T, M, true, NS - 1, +1, NT, 3, 1, 2>(lds, twhr, tid, nold, st);
}

// 2048 points: held to three waves per SIMD, i.e. three 52 KB pencils of 256
// threads per CU in FP64
template <typename T, int L, int NT>
__global__ void __launch_bounds__(NT, L == 2048 ? 3 : 1) k_fused_y_h2(const FusedPass a) {
    using C = cplx<T>;
    constexpr int M = L / 2;
    constexpr int NS = ct::nst(M);
    static_assert(ct::is_pow2(L) && NS >= 2, "two or more radix stages per half-spectrum");
    // outputs per thread of the last inverse stage (reversed radix order)
    constexpr int RL = ct::prad(M, true, NS - 1);
    constexpr int UL = (3 * (M / RL) + NT - 1) / NT;
    // inputs per thread of the first forward stage
    constexpr int R0 = ct::prad(M, false, 0);
    constexpr int U0 = (3 * (M / R0) + NT - 1) / NT;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const int tid = (int)threadIdx.x;
    const int p = (int)xcd_tile(blockIdx.x, gridDim.x);
    const int n = a.n;
    const int kz = p / a.Lx, kx = pair_kx(p - kz * a.Lx, a.Lx);
    C *pen = reinterpret_cast<C *>(a.data) + ((int64_t)kz * a.Lx + kx) * (3 * n);
    // rows past n (the zero padding) read as zero and are not written
    const BufRsrc rp = make_rsrc(pen, (uint32_t)(3 * n) * sizeof(C));
    const PencilProduct<T, L> pr = pencil_product<T, L>(a, kz, kx);
    C acc[UL][RL];
    C xin[U0][R0];
    h2_half<T, L, NT, 0>(lds, a, rp, pr, acc, xin, tid);
    // the even half's last stage has finished reading LDS
    __syncthreads();
    h2_half<T, L, NT, 1>(lds, a, rp, pr, acc, xin, tid);
}

// ---------------- launchers -------------------------------------------------
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
hipError_t launch_fused_y(const FusedPass *d_descs, const int2 *d_map, int tiles, int nthr, size_t lds_bytes,
                          hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fused_y<T>), dim3(tiles), dim3(nthr), lds_bytes, s, d_descs, d_map);
    return hipGetLastError();
}

// Specialised shapes of the x pass: for each power-of-two length two tile
// widths W (columns per tile); NT = W L / 16 threads so each holds 16 complex
// values.  Variant 0 keeps a tile's LDS near 64 KB, variant 1 doubles it;
// variant 2 is the half-LDS kernel on variant 1's tiles, variant 3 the
// half-LDS kernel on tiles twice as wide (lines of 1024 to 4096 points, at
// most 1024 threads holding two or more butterflies each).
static int line_ct_w(int L, bool f32, int variant) {
    int w;
    switch (L) {
    case 64: case 96: case 128: case 160: case 192: case 224: case 256: w = 16; break;
    case 320: case 384: case 448: case 512: w = f32 ? 16 : 8; break;
    case 640: case 768: case 896: case 1024: w = f32 ? 8 : 4; break;
    case 1280: case 1536: case 1792: case 2048: w = f32 ? 4 : 2; break;
    case 4096: w = f32 ? 2 : 1; break;
    default: return 0;
    }
    // the half-LDS kernels (variants 2, 3) exchange half lines: even radices only
    if (variant >= 2 && (L & (L - 1))) return 0;
    if (variant == 3) return L >= 1024 ? 4 * w : 0;
    return variant ? 2 * w : w;
}

int line_ct_shape(int L, size_t csz, int variant, int *W, int *NT) {
    const int w = line_ct_w(L, csz == 8, variant);
    if (!w) return 0;
    *W = w;
    *NT = std::min(1024, w * L / 16);
    return *NT >= 64;
}

#define LINE_CASE(LL, WW)                                                                                             \
    if (a.f.L == LL && W == WW) {                                                                                     \
        if constexpr (ct::is_pow2(LL) && ct::nst(LL) >= 2) {                                                          \
            if (half) {                                                                                               \
                const size_t lh = line_hx_lds(LL, WW, sizeof(cplx<T>));                                               \
                if (dir < 0) hipLaunchKernelGGL((k_line_hx<T, LL, -1, (WW * LL / 16), WW>), dim3(tiles), dim3(WW * LL / 16), lh, s, a); \
                else hipLaunchKernelGGL((k_line_hx<T, LL, +1, (WW * LL / 16), WW>), dim3(tiles), dim3(WW * LL / 16), lh, s, a);       \
                return hipGetLastError();                                                                             \
            }                                                                                                         \
        }                                                                                                             \
        if (dir < 0) hipLaunchKernelGGL((k_line_ct<T, LL, -1, (WW * LL / 16), WW>), dim3(tiles), dim3(WW * LL / 16), lds, s, a); \
        else hipLaunchKernelGGL((k_line_ct<T, LL, +1, (WW * LL / 16), WW>), dim3(tiles), dim3(WW * LL / 16), lds, s, a);       \
        return hipGetLastError();                                                                                     \
    }

// half != 0: the half-LDS kernel (k_line_hx)
template <typename T>
hipError_t launch_line_ct(const LinePass &a, int tiles, int W, int dir, hipStream_t s, int half) {
    if (tiles <= 0) return hipSuccess;
    const size_t lds = line_ct_lds(a.f.L, W, sizeof(cplx<T>));
    if constexpr (sizeof(T) == 4) {
        LINE_CASE(64, 16) LINE_CASE(64, 32) LINE_CASE(128, 16) LINE_CASE(128, 32) LINE_CASE(256, 16) LINE_CASE(256, 32)
        LINE_CASE(512, 16) LINE_CASE(512, 32) LINE_CASE(1024, 8) LINE_CASE(1024, 16) LINE_CASE(2048, 4) LINE_CASE(2048, 8)
        LINE_CASE(4096, 2) LINE_CASE(4096, 4)
        LINE_CASE(384, 16) LINE_CASE(384, 32) LINE_CASE(768, 8) LINE_CASE(768, 16) LINE_CASE(1536, 4) LINE_CASE(1536, 8)
        LINE_CASE(96, 16) LINE_CASE(96, 32) LINE_CASE(160, 16) LINE_CASE(160, 32) LINE_CASE(192, 16) LINE_CASE(192, 32)
        LINE_CASE(224, 16) LINE_CASE(224, 32) LINE_CASE(320, 16) LINE_CASE(320, 32) LINE_CASE(448, 16) LINE_CASE(448, 32)
        LINE_CASE(640, 8) LINE_CASE(640, 16) LINE_CASE(896, 8) LINE_CASE(896, 16) LINE_CASE(1280, 4) LINE_CASE(1280, 8)
        LINE_CASE(1792, 4) LINE_CASE(1792, 8)
    } else {
        LINE_CASE(64, 16) LINE_CASE(64, 32) LINE_CASE(128, 16) LINE_CASE(128, 32) LINE_CASE(256, 16) LINE_CASE(256, 32)
        LINE_CASE(512, 8) LINE_CASE(512, 16) LINE_CASE(1024, 4) LINE_CASE(1024, 8) LINE_CASE(2048, 2) LINE_CASE(2048, 4)
        LINE_CASE(4096, 1) LINE_CASE(4096, 2)
        LINE_CASE(384, 8) LINE_CASE(384, 16) LINE_CASE(768, 4) LINE_CASE(768, 8) LINE_CASE(1536, 2) LINE_CASE(1536, 4)
        LINE_CASE(96, 16) LINE_CASE(96, 32) LINE_CASE(160, 16) LINE_CASE(160, 32) LINE_CASE(192, 16) LINE_CASE(192, 32)
        LINE_CASE(224, 16) LINE_CASE(224, 32) LINE_CASE(320, 8) LINE_CASE(320, 16) LINE_CASE(448, 8) LINE_CASE(448, 16)
        LINE_CASE(640, 4) LINE_CASE(640, 8) LINE_CASE(896, 4) LINE_CASE(896, 8) LINE_CASE(1280, 2) LINE_CASE(1280, 4)
        LINE_CASE(1792, 2) LINE_CASE(1792, 4)
    }
    return hipErrorInvalidValue;
}
#undef LINE_CASE

// variant 3: the half-LDS kernel with 1024 threads on the wide tiles
#define LINE_CASE_W(LL, WW)                                                                                           \
    if (a.f.L == LL && W == WW) {                                                                                     \
        const size_t lh = line_hx_lds(LL, WW, sizeof(cplx<T>));                                                       \
        if (dir < 0) hipLaunchKernelGGL((k_line_hx<T, LL, -1, 1024, WW>), dim3(tiles), dim3(1024), lh, s, a);        \
        else hipLaunchKernelGGL((k_line_hx<T, LL, +1, 1024, WW>), dim3(tiles), dim3(1024), lh, s, a);                \
        return hipGetLastError();                                                                                     \
    }

template <typename T>
hipError_t launch_line_wide(const LinePass &a, int tiles, int W, int dir, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    if constexpr (sizeof(T) == 4) {
        LINE_CASE_W(1024, 32) LINE_CASE_W(2048, 16) LINE_CASE_W(4096, 8)
    } else {
        LINE_CASE_W(1024, 16) LINE_CASE_W(2048, 8) LINE_CASE_W(4096, 4)
    }
    return hipErrorInvalidValue;
}
#undef LINE_CASE_W

#define LINE_CASE_WB(LL, WW)                                                                                          \
    if (L == LL && W == WW) {                                                                                         \
        const size_t lh = line_hx_lds(LL, WW, sizeof(cplx<T>));                                                       \
        if (dir < 0) hipLaunchKernelGGL((k_line_hx_b<T, LL, -1, 1024, WW>), dim3(tiles), dim3(1024), lh, s, d, map); \
        else hipLaunchKernelGGL((k_line_hx_b<T, LL, +1, 1024, WW>), dim3(tiles), dim3(1024), lh, s, d, map);         \
        return hipGetLastError();                                                                                     \
    }

// variant 3 over many geometries of the same length
template <typename T>
hipError_t launch_line_wide_b(const LinePass *d, const int2 *map, int tiles, int L, int W, int dir, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    if constexpr (sizeof(T) == 4) {
        LINE_CASE_WB(1024, 32) LINE_CASE_WB(2048, 16) LINE_CASE_WB(4096, 8)
    } else {
        LINE_CASE_WB(1024, 16) LINE_CASE_WB(2048, 8) LINE_CASE_WB(4096, 4)
    }
    return hipErrorInvalidValue;
}
#undef LINE_CASE_WB

size_t line_ct_lds(int L, int W, size_t csz) { return (size_t)W * ct::lds_pitch(L, W, (int)csz) * csz; }
size_t line_hx_lds(int L, int W, size_t csz) { return (size_t)W * ct::lds_pitch(L / 2, W, (int)csz) * csz; }
size_t fused_ct_lds(int L, size_t csz) { return (size_t)3 * ct::lds_pitch(L, 3, (int)csz) * csz; }

int fused_ct_threads(int L, size_t csz) {
    switch (L) {
    case 64: return 64;
    case 128: return 64;
    case 256: return 64;
    case 96: case 160: case 192: case 224: case 320: return 64;
    case 384: case 448: case 640: return 128;
    case 512: return 128;
    case 896: return 192;
    case 768: return 256;
    case 1024: case 1280: return 256;
    case 1536: return 512;
    case 1792: return 384;
    case 2048: return csz == 8 ? 256 : 384;
    case 4096: return 768;
    default: return 0;
    }
}

template <typename T>
hipError_t launch_fused_ct(const FusedPass &a, hipStream_t s) {
    if (a.npos <= 0) return hipSuccess;
    const size_t lds = fused_ct_lds(a.f.L, sizeof(cplx<T>));
#define FCASE(LL, NTT)                                                                                                \
    case LL:                                                                                                          \
        hipLaunchKernelGGL((k_fused_y_ct<T, LL, NTT>), dim3(a.npos), dim3(NTT), lds, s, a);                         \
        break;
    // one pencil per workgroup; 2048 points: 256 threads in FP32 (three
    // workgroups per CU fill the LDS), 384 in FP64 (one per CU)
    switch (a.f.L) {
        FCASE(64, 64) FCASE(128, 64) FCASE(256, 64) FCASE(512, 128) FCASE(1024, 256)
        FCASE(2048, (sizeof(T) == 4 ? 256 : 384)) FCASE(4096, 768)
        FCASE(384, 128) FCASE(768, 256) FCASE(1536, 512)
        FCASE(96, 64) FCASE(160, 64) FCASE(192, 64) FCASE(224, 64) FCASE(320, 64) FCASE(448, 128) FCASE(640, 128)
        FCASE(896, 192) FCASE(1280, 256) FCASE(1792, 384)
    default: return hipErrorInvalidValue;
    }
#undef FCASE
    return hipGetLastError();
}

// Persistent fused pass (k_fused_y_pf): as many workgroups as fit on the
// device at once (a multiple of 8, so every XCD gets the same number), each
// walking pencils with the next one's loads in flight.
template <typename T, int L, int NT, bool EARLY, int MINW = 1>
hipError_t launch_fused_pf_k(const FusedPass &a, hipStream_t s) {
    const size_t lds = fused_ct_lds(L, sizeof(cplx<T>));
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&k_fused_y_pf<T, L, NT, EARLY, MINW>), NT, lds);
    if (e != hipSuccess) return e;
    int G = std::max(1, per_cu) * std::max(1, ncu);
    G = std::max(8, G - G % 8);
    G = std::min(G, a.npos);
    hipLaunchKernelGGL((k_fused_y_pf<T, L, NT, EARLY, MINW>), dim3(G), dim3(NT), lds, s, a);
    return hipGetLastError();
}

// k_fused_y_pt: the pencil and the root table in LDS, a resident grid as
// for k_fused_y_pf
template <typename T, int L, int NT, bool EARLY>
hipError_t launch_fused_pt_k(const FusedPass &a, hipStream_t s) {
    const size_t lds = fused_ct_lds(L, sizeof(cplx<T>)) + (size_t)L * sizeof(cplx<T>);
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&k_fused_y_pt<T, L, NT, EARLY>),
                                                         NT, lds);
    if (e != hipSuccess) return e;
    int G = std::max(1, per_cu) * std::max(1, ncu);
    G = std::max(8, G - G % 8);
    G = std::min(G, a.npos);
    hipLaunchKernelGGL((k_fused_y_pt<T, L, NT, EARLY>), dim3(G), dim3(NT), lds, s, a);
    return hipGetLastError();
}

// variant 2: k_fused_y_cr (one pencil per workgroup, waves rotated);
// variant 3: k_fused_y_pf (persistent, next pencil's loads in flight; in
// FP32 with one radix-16 butterfly per thread, 384 threads for 2048 points,
// and the tensor fetched at the product, which keeps it under 168 VGPRs)
// variant 4: the persistent kernel with 256 threads held to three waves per
// SIMD (2048-point FP32 pencils)
// variant 5: k_fused_y_pt (persistent, twiddles from a root table in LDS)
// variant 6: k_fused_y_h2 (two half-spectra through an LDS pencil of Ly/2)
int fused_pf_available(int L, int var) {
    if (var == 2) return L >= 256 && L <= 4096 && (L & (L - 1)) == 0 && fused_ct_threads(L, 8) > 64;
    if (var == 4) return L == 2048;
    if (var == 6) return L == 1024 || L == 2048 || L == 4096;
    return (var == 3 || var == 5) && (L == 1024 || L == 2048);
}

template <typename T>
hipError_t launch_fused_pf(const FusedPass &a, int var, hipStream_t s) {
    if (a.npos <= 0) return hipSuccess;
    if (var == 2) {
        const size_t lds = fused_ct_lds(a.f.L, sizeof(cplx<T>));
#define RCASE(LL, NTT)                                                                                                \
    case LL:                                                                                                          \
        hipLaunchKernelGGL((k_fused_y_cr<T, LL, NTT>), dim3(a.npos), dim3(NTT), lds, s, a);                         \
        break;
        switch (a.f.L) {
            RCASE(512, 128) RCASE(1024, 256) RCASE(2048, (sizeof(T) == 4 ? 256 : 384)) RCASE(4096, 768)
        default: return hipErrorInvalidValue;
        }
#undef RCASE
        return hipGetLastError();
    }
    constexpr bool F32 = sizeof(T) == 4;
    if (var == 6) {
        if (!a.twh) return hipErrorInvalidValue;
        const size_t lds = fused_ct_lds(a.f.L / 2, sizeof(cplx<T>));
#define HCASE2(LL, NTT)                                                                                               \
    case LL:                                                                                                          \
        hipLaunchKernelGGL((k_fused_y_h2<T, LL, NTT>), dim3(a.npos), dim3(NTT), lds, s, a);                         \
        break;
        switch (a.f.L) {
            HCASE2(1024, 128) HCASE2(2048, 256) HCASE2(4096, (F32 ? 256 : 384))
        default: return hipErrorInvalidValue;
        }
#undef HCASE2
        return hipGetLastError();
    }
    if (var == 5) {
        if (a.f.L == 2048) return launch_fused_pt_k<T, 2048, (F32 ? 256 : 384), false>(a, s);
        if (a.f.L == 1024) return launch_fused_pt_k<T, 1024, 256, true>(a, s);
        return hipErrorInvalidValue;
    }
    if (var == 4) {
        if (a.f.L != 2048) return hipErrorInvalidValue;
        if constexpr (F32) return launch_fused_pf_k<T, 2048, 256, false, 3>(a, s);
        else return launch_fused_pf_k<T, 2048, 384, false>(a, s);
    }
    switch (a.f.L) {
    case 1024: return launch_fused_pf_k<T, 1024, 256, F32>(a, s);
    case 2048: return launch_fused_pf_k<T, 2048, 384, false>(a, s);
    default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_fused_pf<float>(const FusedPass &, int, hipStream_t);
template hipError_t launch_fused_pf<double>(const FusedPass &, int, hipStream_t);

// threads of the register-resident fused pass: one radix-16 butterfly per
// thread and stage, rounded up to whole waves
int fused_hx_threads(int L) {
    switch (L) {
    case 256: return 64;
    case 512: return 128;
    case 1024: return 192;
    case 2048: return 384;
    default: return 0;
    }
}
size_t fused_hx_lds(int L, size_t csz) { return (size_t)3 * ct::lds_pitch(L / 2, 3, (int)csz) * csz; }

template <typename T>
hipError_t launch_fused_hx(const FusedPass &a, hipStream_t s) {
    if (a.npos <= 0) return hipSuccess;
    const size_t lds = fused_hx_lds(a.f.L, sizeof(cplx<T>));
#define HCASE(LL, NTT)                                                                                                \
    case LL:                                                                                                          \
        hipLaunchKernelGGL((k_fused_y_hx<T, LL, NTT>), dim3(a.npos), dim3(NTT), lds, s, a);                         \
        break;
    switch (a.f.L) {
        HCASE(256, 64) HCASE(512, 128) HCASE(1024, 192) HCASE(2048, 384)
    default: return hipErrorInvalidValue;
    }
#undef HCASE
    return hipGetLastError();
}
template hipError_t launch_fused_hx<float>(const FusedPass &, hipStream_t);
template hipError_t launch_fused_hx<double>(const FusedPass &, hipStream_t);

// grouped launch of the specialised fused kernel (descriptor table + tile
// map; every geometry in the group has the same transform length)
template <typename T>
hipError_t launch_fused_ct_b(const FusedPass *d, const int2 *map, int tiles, int L, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    const size_t lds = fused_ct_lds(L, sizeof(cplx<T>));
#define FB(LL, NTT)                                                                                                   \
    case LL:                                                                                                          \
        hipLaunchKernelGGL((k_fused_y_ct_b<T, LL, NTT>), dim3(tiles), dim3(NTT), lds, s, d, map);                   \
        break;
    switch (L) {
        FB(64, 64) FB(128, 64) FB(256, 64) FB(512, 128) FB(1024, 256) FB(2048, (sizeof(T) == 4 ? 256 : 384)) FB(4096, 768)
        FB(384, 128) FB(768, 256) FB(1536, 512)
        FB(96, 64) FB(160, 64) FB(192, 64) FB(224, 64) FB(320, 64) FB(448, 128) FB(640, 128) FB(896, 192)
        FB(1280, 256) FB(1792, 384)
    default: return hipErrorInvalidValue;
    }
#undef FB
    return hipGetLastError();
}

// Grouped x pass in any of the four variants (as launch_line_ct /
// launch_line_wide for one geometry).
template <typename T>
hipError_t launch_line_var_b(const LinePass *d, const int2 *map, int tiles, int L, int W, int dir, int var,
                             hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    if (var == 3) return launch_line_wide_b<T>(d, map, tiles, L, W, dir, s);
    const size_t lds = var == 2 ? line_hx_lds(L, W, sizeof(cplx<T>)) : line_ct_lds(L, W, sizeof(cplx<T>));
#define LVB(LL, WW)                                                                                                   \
    if (L == LL && W == WW) {                                                                                         \
        constexpr int NTT = WW * LL / 16;                                                                             \
        if constexpr (ct::is_pow2(LL) && ct::nst(LL) >= 2) {                                                          \
            if (var == 2) {                                                                                           \
                if (dir < 0) hipLaunchKernelGGL((k_line_hx_b<T, LL, -1, NTT, WW>), dim3(tiles), dim3(NTT), lds, s, d, map); \
                else hipLaunchKernelGGL((k_line_hx_b<T, LL, +1, NTT, WW>), dim3(tiles), dim3(NTT), lds, s, d, map);   \
                return hipGetLastError();                                                                             \
            }                                                                                                         \
        }                                                                                                             \
        if (dir < 0) hipLaunchKernelGGL((k_line_ct_b<T, LL, -1, NTT, WW>), dim3(tiles), dim3(NTT), lds, s, d, map);  \
        else hipLaunchKernelGGL((k_line_ct_b<T, LL, +1, NTT, WW>), dim3(tiles), dim3(NTT), lds, s, d, map);           \
        return hipGetLastError();                                                                                     \
    }
    if constexpr (sizeof(T) == 4) {
        LVB(64, 16) LVB(64, 32) LVB(128, 16) LVB(128, 32) LVB(256, 16) LVB(256, 32) LVB(512, 16) LVB(512, 32)
        LVB(1024, 8) LVB(1024, 16) LVB(2048, 4) LVB(2048, 8) LVB(4096, 2) LVB(4096, 4)
        LVB(384, 16) LVB(384, 32) LVB(768, 8) LVB(768, 16) LVB(1536, 4) LVB(1536, 8)
        LVB(96, 16) LVB(96, 32) LVB(160, 16) LVB(160, 32) LVB(192, 16) LVB(192, 32) LVB(224, 16) LVB(224, 32)
        LVB(320, 16) LVB(320, 32) LVB(448, 16) LVB(448, 32) LVB(640, 8) LVB(640, 16) LVB(896, 8) LVB(896, 16)
        LVB(1280, 4) LVB(1280, 8) LVB(1792, 4) LVB(1792, 8)
    } else {
        LVB(64, 16) LVB(64, 32) LVB(128, 16) LVB(128, 32) LVB(256, 16) LVB(256, 32) LVB(512, 8) LVB(512, 16)
        LVB(1024, 4) LVB(1024, 8) LVB(2048, 2) LVB(2048, 4) LVB(4096, 1) LVB(4096, 2)
        LVB(384, 8) LVB(384, 16) LVB(768, 4) LVB(768, 8) LVB(1536, 2) LVB(1536, 4)
        LVB(96, 16) LVB(96, 32) LVB(160, 16) LVB(160, 32) LVB(192, 16) LVB(192, 32) LVB(224, 16) LVB(224, 32)
        LVB(320, 8) LVB(320, 16) LVB(448, 8) LVB(448, 16) LVB(640, 4) LVB(640, 8) LVB(896, 4) LVB(896, 8)
        LVB(1280, 2) LVB(1280, 4) LVB(1792, 2) LVB(1792, 4)
    }
#undef LVB
    return hipErrorInvalidValue;
}

// Grouped fused y pass: variant 0 LDS-resident pencils, 1 register-resident,
// 2 LDS-resident with rotated waves (the persistent variant has no grouped
// form).
template <typename T>
hipError_t launch_fused_var_b(const FusedPass *d, const int2 *map, int tiles, int L, int var, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    if (var == 0) return launch_fused_ct_b<T>(d, map, tiles, L, s);
    if (var == 1) {
        const size_t lds = fused_hx_lds(L, sizeof(cplx<T>));
        switch (L) {
        case 256: hipLaunchKernelGGL((k_fused_y_hx_b<T, 256, 64>), dim3(tiles), dim3(64), lds, s, d, map); break;
        case 512: hipLaunchKernelGGL((k_fused_y_hx_b<T, 512, 128>), dim3(tiles), dim3(128), lds, s, d, map); break;
        case 1024: hipLaunchKernelGGL((k_fused_y_hx_b<T, 1024, 192>), dim3(tiles), dim3(192), lds, s, d, map); break;
        case 2048: hipLaunchKernelGGL((k_fused_y_hx_b<T, 2048, 384>), dim3(tiles), dim3(384), lds, s, d, map); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (var == 2) {
        const size_t lds = fused_ct_lds(L, sizeof(cplx<T>));
        switch (L) {
        case 512: hipLaunchKernelGGL((k_fused_y_cr_b<T, 512, 128>), dim3(tiles), dim3(128), lds, s, d, map); break;
        case 1024: hipLaunchKernelGGL((k_fused_y_cr_b<T, 1024, 256>), dim3(tiles), dim3(256), lds, s, d, map); break;
        case 2048:
            hipLaunchKernelGGL((k_fused_y_cr_b<T, 2048, (sizeof(T) == 4 ? 256 : 384)>), dim3(tiles),
                               dim3(sizeof(T) == 4 ? 256 : 384), lds, s, d, map);
            break;
        case 4096: hipLaunchKernelGGL((k_fused_y_cr_b<T, 4096, 768>), dim3(tiles), dim3(768), lds, s, d, map); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}
template hipError_t launch_line_var_b<float>(const LinePass *, const int2 *, int, int, int, int, int, hipStream_t);
template hipError_t launch_line_var_b<double>(const LinePass *, const int2 *, int, int, int, int, int, hipStream_t);
template hipError_t launch_fused_var_b<float>(const FusedPass *, const int2 *, int, int, int, hipStream_t);
template hipError_t launch_fused_var_b<double>(const FusedPass *, const int2 *, int, int, int, hipStream_t);

template hipError_t launch_fused_ct_b<float>(const FusedPass *, const int2 *, int, int, hipStream_t);
template hipError_t launch_fused_ct_b<double>(const FusedPass *, const int2 *, int, int, hipStream_t);
template hipError_t launch_line_pass<float>(const LinePass *, const int2 *, int, int, size_t, int, bool, hipStream_t);
template hipError_t launch_line_pass<double>(const LinePass *, const int2 *, int, int, size_t, int, bool, hipStream_t);
template hipError_t launch_fused_y<float>(const FusedPass *, const int2 *, int, int, size_t, hipStream_t);
template hipError_t launch_fused_y<double>(const FusedPass *, const int2 *, int, int, size_t, hipStream_t);
template hipError_t launch_line_ct<float>(const LinePass &, int, int, int, hipStream_t, int);
template hipError_t launch_line_ct<double>(const LinePass &, int, int, int, hipStream_t, int);
template hipError_t launch_line_wide<float>(const LinePass &, int, int, int, hipStream_t);
template hipError_t launch_line_wide<double>(const LinePass &, int, int, int, hipStream_t);
template hipError_t launch_line_wide_b<float>(const LinePass *, const int2 *, int, int, int, int, hipStream_t);
template hipError_t launch_line_wide_b<double>(const LinePass *, const int2 *, int, int, int, int, hipStream_t);
template hipError_t launch_fused_ct<float>(const FusedPass &, hipStream_t);
template hipError_t launch_fused_ct<double>(const FusedPass &, hipStream_t);

}  // namespace mmx
