// Compile-time z passes for power-of-two Lz = 2N: each real z-line of a cell
// column is folded into a complex line of length N (even samples real, odd
// samples imaginary), transformed, and unfolded into the Lz/2+1 half
// spectrum; the inverse folds the half spectrum back, transforms and reads
// the even/odd samples out.  Lines are the 3 components of P cell columns.
#pragma once
#include "kernels.hpp"
#include "fft_engine.hpp"
#include "zepi.hpp"

namespace mmx {

namespace {
// LDS pitch of a folded z line; the tile interleaves the three components of
// each of its 3 zcols(N) columns, and the shift keeps the lanes of one
// 128-byte LDS cycle in distinct banks in the transform's exchanges
constexpr int zpitch(int N) {
    return N < 16 ? N + 1 : ct::line_len(N) + (N == 32 ? 9 : N == 64 ? 7 : N == 128 ? 3 : 11);
}
constexpr int zcols(int N) { return N >= 1024 ? 1 : 1024 / N; }   // P: ~3072 complex per tile
constexpr int zthreads(int N) { return 256; }
}  // namespace

// Lines of a tile past its last cell column (the grid's last tile) are
// transformed like the others but never stored.
//
// unfold: X[k] = E[k] + W^k O[k], E = (Z[k] + conj Z[N-k])/2, O = (Z[k] - conj Z[N-k])/(2i),
// W = exp(-2 pi i / 2N); since E[N-k] = conj E[k] and O[N-k] = conj O[k], one
// pair (Z[k], Z[N-k]) gives X[k] and X[N-k].  Written to S1 [kz][pos][c].
template <typename T, int N, int NT, int NL, int PT, typename I = int64_t>
__device__ __forceinline__ void zunfold_store(const cplx<T> *lds, const ZGeom &g, int64_t pos0, int w3,
                                              const cplx<T> *__restrict__ wt, int tid) {
    using C = cplx<T>;
    const I npos3 = (I)g.nx * (I)g.ny * 3;
    C *S1 = reinterpret_cast<C *>(g.S1) + pos0 * 3;
    const T h = T(0.5);
    constexpr int NE = (N / 2 + 1) * NL;
    constexpr int CH = sizeof(T) == 4 ? 8 : 4;
    for (int e0 = 0; e0 < NE; e0 += CH * NT) {
        C w[CH], wm[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = e0 + tid + u * NT;
            if (e < NE) {
                const int k = e / NL;
                w[u] = wt[k];
                wm[u] = wt[N - k];
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = e0 + tid + u * NT;
            if (e < NE) {
                const int k = e / NL, l = e - k * NL;
                const C za = lds[l * PT + sw<N>(k % N)];
                const C zb = lds[l * PT + sw<N>((N - k) % N)];
                const C E = cmake<C>(h * (za.x + zb.x), h * (za.y - zb.y));
                const C O = cmake<C>(h * (za.y + zb.y), -h * (za.x - zb.x));
                if (l < w3) {
                    S1[k * npos3 + l] = cmake<C>(E.x + w[u].x * O.x - w[u].y * O.y, E.y + w[u].x * O.y + w[u].y * O.x);
                    if (2 * k != N)
                        S1[(N - k) * npos3 + l] = cmake<C>(E.x + wm[u].x * O.x + wm[u].y * O.y,
                                                           -E.y - wm[u].x * O.y + wm[u].y * O.x);
                }
            }
        }
    }
}

template <typename T, int N, int SRC>
__device__ __forceinline__ void zfwd_ct_body(const ZFwdArgs &a, uint32_t tile) {
    using C = cplx<T>;
    constexpr int NT = zthreads(N), P = zcols(N), NL = 3 * P, PT = zpitch(N);
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const ZGeom &g = a.g;
    const int tid = threadIdx.x;
    const int64_t npos = (int64_t)g.nx * g.ny;
    const int64_t pos0 = (int64_t)tile * P;
    const int wp = (int)min((int64_t)P, npos - pos0);
    const int nz = g.nz;
    const T *src = reinterpret_cast<const T *>(a.src);
    const T *Ms = reinterpret_cast<const T *>(a.Ms);
    const T Ms_s = T(a.Ms_scalar);
    auto ld = [&](int l, int n) -> C {
        const int pl = l / 3, c = l - 3 * pl;
        const int z0 = 2 * n;
        if (pl >= wp || z0 >= nz) return cmake<C>(T(0), T(0));
        const int64_t cell = (pos0 + pl) * nz + z0;
        T re = src[cell * 3 + c], im = T(0);
        if (SRC == SRC_MS_M) re *= ms_at(Ms, Ms_s, cell);
        if (z0 + 1 < nz) {
            im = src[cell * 3 + 3 + c];
            if (SRC == SRC_MS_M) im *= ms_at(Ms, Ms_s, cell + 1);
        }
        return cmake<C>(re, im);
    };
    auto nost = [](int, int, C) {};
    const C *tw = reinterpret_cast<const C *>(g.twh);
    // folded samples occupy slots < ceil(nz/2) <= N/2
    eng_fft_la<T, N, -1, NT, NL, 3, PT, 0, 1, 1>(lds, tw, tid, ld, nost);
    zunfold_store<T, N, NT, NL, PT>(lds, g, pos0, 3 * wp, tw + (N > 1 ? N - 1 : 0), tid);
}

// Epilogue over the tile's cells, two cells per thread at a time: both cells'
// loads are issued before either's arithmetic.  The demag field sample z of
// component c sits in line 3 pl + c, slot z/2, real part for even z; the next
// stage's source is written back to the same place.
template <typename T, int N, int EPI, bool MSV, bool LOC, typename I>
__device__ __forceinline__ void zepi_cells(const ZInvArgs &a, cplx<T> *lds, int64_t pos0, int ncells, bool demag,
                                           Acc4 &acc, int tid) {
    constexpr int NT = zthreads(N), PT = zpitch(N);
    const ZGeom &g = a.g;
    const int nz = g.nz, ny = g.ny;
    auto where = [&](int e, int &pl, int &z, I &cell, int &i, int &j) {
        pl = (int)fdiv((uint32_t)e, g.dnz);
        z = e - pl * nz;
        const I pos = (I)pos0 + (I)pl;
        i = (int)fdiv((uint32_t)pos, g.dny);
        j = (int)(pos - (I)i * (I)ny);
        cell = pos * (I)nz + (I)z;
    };
    auto finish = [&](int pl, int z, const CellIn<T, I> &in) {
        T hd[3] = {T(0), T(0), T(0)};
        if (demag) {
#pragma unroll
            for (int c = 0; c < 3; ++c) hd[c] = reinterpret_cast<const T *>(&lds[(pl * 3 + c) * PT + sw<N>(z >> 1)])[z & 1];
        }
        T srcn[3] = {T(0), T(0), T(0)};
        cell_compute<T, EPI, MSV, LOC>(a, in, hd, acc, srcn);
        if ((EPI == EPI_STAGE || EPI == EPI_TAB) && a.next_r2c) {
#pragma unroll
            for (int c = 0; c < 3; ++c) reinterpret_cast<T *>(&lds[(pl * 3 + c) * PT + sw<N>(z >> 1)])[z & 1] = srcn[c];
        }
    };
    for (int e0 = tid; e0 < ncells; e0 += 2 * NT) {
        const int e1 = e0 + NT;
        const bool two = e1 < ncells;
        int pl0, z0, i0, j0, pl1 = 0, z1 = 0, i1 = 0, j1 = 0;
        I c0, c1 = 0;
        where(e0, pl0, z0, c0, i0, j0);
        CellIn<T, I> in0, in1;
        cell_load<T, EPI, MSV, LOC>(a, c0, i0, j0, z0, in0);
        if (two) {
            where(e1, pl1, z1, c1, i1, j1);
            cell_load<T, EPI, MSV, LOC>(a, c1, i1, j1, z1, in1);
        }
        finish(pl0, z0, in0);
        if (two) finish(pl1, z1, in1);
    }
}

// Tiles of the z-inverse pass with the exchange epilogue.  Linear runs of P
// positions (ygrp = 0), or P positions of one x row with the tiles ordered
// by groups of ygrp y-blocks, x fastest within a group: the tiles that hold a
// cell's x neighbours (one x row apart) then run at the same time as it, so
// the neighbours' m rows come from L2 instead of being fetched again.
// Returns the tile's first position and width (0 for the padding tiles of a
// last, incomplete group).
__host__ __device__ inline int ztile_count(int nx, int ny, int P, int ygrp) {
    if (ygrp <= 0) return (int)(((int64_t)nx * ny + P - 1) / P);
    const int ty = (ny + P - 1) / P;
    return ((ty + ygrp - 1) / ygrp) * nx * ygrp;
}

__device__ __forceinline__ void ztile(const ZGeom &g, int P, uint32_t blk, int64_t &pos0, int &wp) {
    const int64_t npos = (int64_t)g.nx * g.ny;
    if (g.ygrp <= 0) {
        pos0 = (int64_t)blk * P;
        wp = (int)min((int64_t)P, npos - pos0);
        return;
    }
    const int ty = (g.ny + P - 1) / P, G = g.ygrp;
    const uint32_t per = (uint32_t)g.nx * (uint32_t)G;
    const uint32_t yo = blk / per, rem = blk - yo * per;
    const int x = (int)(rem / (uint32_t)G), yb = (int)(yo * G + (rem - (uint32_t)x * G));
    if (yb >= ty) {
        pos0 = 0;
        wp = 0;
        return;
    }
    pos0 = (int64_t)x * g.ny + (int64_t)yb * P;
    wp = min(P, g.ny - yb * P);
}

// I: type of the cell and S1 indices (int when they fit, see CellIn)
template <typename T, int N, int EPI, bool LOC, typename I = int64_t>
__device__ __forceinline__ void zinv_ct_body(const ZInvArgs &a, uint32_t blk) {
    using C = cplx<T>;
    constexpr int NT = zthreads(N), P = zcols(N), NL = 3 * P, PT = zpitch(N);
    // slots of the folded line that can hold cells: ceil(nz/2) <= N/2; the
    // transforms skip the upper half when they have two or more stages
    constexpr bool HALF = ct::nst(N) >= 2;
    constexpr int NH = HALF ? N / 2 : N;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const ZGeom &g = a.g;
    const int tid = threadIdx.x;
    const int64_t npos = (int64_t)g.nx * g.ny;
    int64_t pos0;
    int wp;
    ztile(g, P, blk, pos0, wp);
    const int w3 = 3 * wp;
    const int nz = g.nz, ny = g.ny;
    // a padding tile (wp = 0) loads and stores nothing but still takes part
    // in the block reductions below
    const bool demag = (a.terms & 1u) != 0 && wp > 0;
    const C *tw = reinterpret_cast<const C *>(g.twh);
    const C *wt = tw + (N > 1 ? N - 1 : 0);
    if (demag) {
        // 1. half spectra X[k], X[N-k] of the tile's lines (DC and Nyquist
        //    real), folded at once:
        //    Z[k] = (X[k] + conj X[N-k]) + i conj(W^k) (X[k] - conj X[N-k])
        //    Loads of CH iterations are issued before their arithmetic.
        const I npos3 = (I)npos * 3;
        const C *S1 = reinterpret_cast<const C *>(g.S1) + pos0 * 3;
        constexpr int NE = (N / 2 + 1) * NL;
        constexpr int CH = sizeof(T) == 4 ? 8 : 4;
        for (int e0 = 0; e0 < NE; e0 += CH * NT) {
            C xk[CH], xm[CH], wk[CH], wm[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int e = e0 + tid + u * NT;
                if (e < NE) {
                    const int k = e / NL, l = e - k * NL;
                    const int lc = min(l, w3 - 1);
                    xk[u] = S1[(I)k * npos3 + (I)lc];
                    xm[u] = S1[(I)(N - k) * npos3 + (I)lc];
                    wk[u] = wt[k];
                    wm[u] = wt[N - k];
                }
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int e = e0 + tid + u * NT;
                if (e < NE) {
                    const int k = e / NL, l = e - k * NL;
                    C *b = lds + l * PT;
                    if (k == 0) {
                        const C x0 = cmake<C>(xk[u].x, T(0)), xn = cmake<C>(xm[u].x, T(0));
                        const C s = cmake<C>(x0.x + xn.x, x0.y - xn.y), d = cmake<C>(x0.x - xn.x, x0.y + xn.y);
                        b[0] = cmake<C>(s.x - d.y, s.y + d.x);
                    } else {
                        const C xa = xk[u], xb = xm[u];
                        {
                            const C s = cmake<C>(xa.x + xb.x, xa.y - xb.y), d = cmake<C>(xa.x - xb.x, xa.y + xb.y);
                            // i conj(w) d
                            const C w = wk[u];
                            const C cd = cmake<C>(w.x * d.x + w.y * d.y, w.x * d.y - w.y * d.x);
                            b[sw<N>(k)] = cmake<C>(s.x - cd.y, s.y + cd.x);
                        }
                        if (2 * k != N) {
                            const C s = cmake<C>(xb.x + xa.x, xb.y - xa.y), d = cmake<C>(xb.x - xa.x, xb.y + xa.y);
                            const C w = wm[u];
                            const C cd = cmake<C>(w.x * d.x + w.y * d.y, w.x * d.y - w.y * d.x);
                            b[sw<N>(N - k)] = cmake<C>(s.x - cd.y, s.y + cd.x);
                        }
                    }
                }
            }
        }
        __syncthreads();
        auto nold = [](int, int) { return C(); };
        auto nost = [](int, int, C) {};
        eng_fft_la<T, N, +1, NT, NL, 3, PT, 1, 1, HALF ? 2 : 0>(lds, tw, tid, nold, nost);
    }
    // 2. epilogue per cell; demag field sample z of component c sits in line
    //    3 pl + c, slot z/2, real part for even z
    Acc4 acc;
    const int ncells = wp * nz;
    if (a.Ms) zepi_cells<T, N, EPI, true, LOC, I>(a, lds, pos0, ncells, demag, acc, tid);
    else zepi_cells<T, N, EPI, false, LOC, I>(a, lds, pos0, ncells, demag, acc, tid);
    if (EPI == EPI_HEFF && a.epart) block_energy(acc.v[0], acc.v[1], reinterpret_cast<double *>(smem), a.epart + 2 * (int64_t)blk, tid);
    if (EPI == EPI_TAB && a.tab_last) block_max(acc.v[0], reinterpret_cast<double *>(smem), a.epart + 2 * (int64_t)blk, tid);
    if (EPI == EPI_BB) block_bb(acc, reinterpret_cast<double *>(smem), a.bb_part + 4 * (int64_t)blk, tid);
    if ((EPI == EPI_STAGE || EPI == EPI_TAB) && a.next_r2c && wp > 0) {
        // 3. the next stage's source, already folded in LDS: clear the slots
        //    between the last cell and the transform's input half, then
        //    transform forward
        const int n0 = (nz + 1) / 2;
        for (int e = tid; e < (NH - n0) * w3; e += NT) {
            const int k = n0 + e / w3, l = e - (k - n0) * w3;
            lds[l * PT + sw<N>(k)] = cmake<C>(T(0), T(0));
        }
        if (nz & 1) {
            for (int l = tid; l < w3; l += NT) reinterpret_cast<T *>(&lds[l * PT + sw<N>(nz / 2)])[1] = T(0);
        }
        __syncthreads();
        auto nold = [](int, int) { return C(); };
        auto nost = [](int, int, C) {};
        eng_fft_la<T, N, -1, NT, NL, 3, PT, 1, 1, HALF ? 1 : 0>(lds, tw, tid, nold, nost);
        zunfold_store<T, N, NT, NL, PT, I>(lds, g, pos0, w3, wt, tid);
    }
}

template <typename T, int N, int SRC>
__global__ void __launch_bounds__(zthreads(N)) k_zfwd_ct(const ZFwdArgs a) {
    zfwd_ct_body<T, N, SRC>(a, xcd_tile(blockIdx.x, gridDim.x));
}

template <typename T, int N, int SRC>
__global__ void __launch_bounds__(zthreads(N)) k_zfwd_ct_b(const ZFwdArgs *__restrict__ d, const int2 *__restrict__ map) {
    const int2 e = map[xcd_tile(blockIdx.x, gridDim.x)];
    zfwd_ct_body<T, N, SRC>(d[e.x], (uint32_t)e.y);
}

// LOC: the plan carries DMI, anisotropy or spin-transfer torque (a separate
// instantiation keeps the plain exchange epilogue free of those registers).
// The FP64 RK4-stage form without local terms is held to three waves per
// SIMD (168 VGPRs; it spills 20 of its 191 and still runs 7% faster than at
// two waves); the other forms would spill far more.
// I32: cell and S1 indices in 32 bits (the host sets ZInvArgs::i32 when
// every index fits); used by the RK4-stage forms, whose epilogue it makes
// 4-5% faster in FP32 (the h_eff form measured no faster, in FP64 slower).
template <typename T, int N, int EPI, bool LOC, bool I32 = false>
__global__ void __launch_bounds__(zthreads(N), (sizeof(T) == 8 && EPI == EPI_STAGE && !LOC) ? 3 : 1)
k_zinv_ct(const ZInvArgs a) {
    if constexpr (I32) zinv_ct_body<T, N, EPI, LOC, int>(a, xcd_tile(blockIdx.x, gridDim.x));
    else zinv_ct_body<T, N, EPI, LOC>(a, xcd_tile(blockIdx.x, gridDim.x));
}

template <typename T, int N, int EPI>
__global__ void __launch_bounds__(zthreads(N)) k_zinv_ct_b(const ZInvArgs *__restrict__ d, const int2 *__restrict__ map) {
    const int2 e = map[xcd_tile(blockIdx.x, gridDim.x)];
    zinv_ct_body<T, N, EPI, false>(d[e.x], (uint32_t)e.y);   // batch plans carry no local terms
}

// ---------------- launches of one folded length N --------------------------
template <typename T, int NN>
hipError_t zfwd_launch_n(const ZFwdArgs &a, int src_mode, size_t lds, hipStream_t s) {
    const int tiles = (int)(((int64_t)a.g.nx * a.g.ny + zcols(NN) - 1) / zcols(NN));
    if (src_mode == SRC_MS_M) hipLaunchKernelGGL((k_zfwd_ct<T, NN, SRC_MS_M>), dim3(tiles), dim3(zthreads(NN)), lds, s, a);
    else hipLaunchKernelGGL((k_zfwd_ct<T, NN, SRC_RAW>), dim3(tiles), dim3(zthreads(NN)), lds, s, a);
    return hipGetLastError();
}

template <typename T, int NN>
hipError_t zinv_launch_n(const ZInvArgs &a, int epi, size_t lds, hipStream_t s) {
    const int tiles = ztile_count(a.g.nx, a.g.ny, zcols(NN), a.g.ygrp);
    const bool loc = a.dmi_kind != 0 || a.ku_pref != 0.0 || a.stt_pref != 0.0;
#define ZL(E, L) hipLaunchKernelGGL((k_zinv_ct<T, NN, E, L>), dim3(tiles), dim3(zthreads(NN)), lds, s, a)
#define ZL32(E, L) hipLaunchKernelGGL((k_zinv_ct<T, NN, E, L, true>), dim3(tiles), dim3(zthreads(NN)), lds, s, a)
    if (epi == EPI_HEFF && loc) ZL(EPI_HEFF, true);
    else if (epi == EPI_HEFF) ZL(EPI_HEFF, false);
    else if (epi == EPI_STAGE && loc && a.i32) ZL32(EPI_STAGE, true);
    else if (epi == EPI_STAGE && loc) ZL(EPI_STAGE, true);
    else if (epi == EPI_STAGE && a.i32) ZL32(EPI_STAGE, false);
    else if (epi == EPI_STAGE) ZL(EPI_STAGE, false);
    else if (epi == EPI_TAB && loc) ZL(EPI_TAB, true);
    else if (epi == EPI_TAB) ZL(EPI_TAB, false);
    else if (epi == EPI_BB) ZL(EPI_BB, true);
    else ZL(EPI_ADJ, false);
#undef ZL32
#undef ZL
    return hipGetLastError();
}

template <typename T, int NN>
hipError_t zfwd_b_launch_n(const ZFwdArgs *d, const int2 *map, int tiles, int src_mode, size_t lds, hipStream_t s) {
    if (src_mode == SRC_MS_M) hipLaunchKernelGGL((k_zfwd_ct_b<T, NN, SRC_MS_M>), dim3(tiles), dim3(zthreads(NN)), lds, s, d, map);
    else hipLaunchKernelGGL((k_zfwd_ct_b<T, NN, SRC_RAW>), dim3(tiles), dim3(zthreads(NN)), lds, s, d, map);
    return hipGetLastError();
}

template <typename T, int NN>
hipError_t zinv_b_launch_n(const ZInvArgs *d, const int2 *map, int tiles, int epi, size_t lds, hipStream_t s) {
    if (epi == EPI_HEFF) hipLaunchKernelGGL((k_zinv_ct_b<T, NN, EPI_HEFF>), dim3(tiles), dim3(zthreads(NN)), lds, s, d, map);
    else if (epi == EPI_STAGE) hipLaunchKernelGGL((k_zinv_ct_b<T, NN, EPI_STAGE>), dim3(tiles), dim3(zthreads(NN)), lds, s, d, map);
    else hipLaunchKernelGGL((k_zinv_ct_b<T, NN, EPI_ADJ>), dim3(tiles), dim3(zthreads(NN)), lds, s, d, map);
    return hipGetLastError();
}

// The launches of a list of folded lengths; hipErrorInvalidValue when N is
// not in the list.  Each translation unit instantiates its own list, so the
// lengths compile in parallel.
template <typename T, int... Ns> struct ZctLengths {
    static hipError_t fwd(int N, const ZFwdArgs &a, int src_mode, size_t lds, hipStream_t s) {
        hipError_t r = hipErrorInvalidValue;
        (void)((N == Ns && ((r = zfwd_launch_n<T, Ns>(a, src_mode, lds, s)), true)) || ...);
        return r;
    }
    static hipError_t inv(int N, const ZInvArgs &a, int epi, size_t lds, hipStream_t s) {
        hipError_t r = hipErrorInvalidValue;
        (void)((N == Ns && ((r = zinv_launch_n<T, Ns>(a, epi, lds, s)), true)) || ...);
        return r;
    }
    static hipError_t fwd_b(int N, const ZFwdArgs *d, const int2 *map, int tiles, int src_mode, size_t lds, hipStream_t s) {
        hipError_t r = hipErrorInvalidValue;
        (void)((N == Ns && ((r = zfwd_b_launch_n<T, Ns>(d, map, tiles, src_mode, lds, s)), true)) || ...);
        return r;
    }
    static hipError_t inv_b(int N, const ZInvArgs *d, const int2 *map, int tiles, int epi, size_t lds, hipStream_t s) {
        hipError_t r = hipErrorInvalidValue;
        (void)((N == Ns && ((r = zinv_b_launch_n<T, Ns>(d, map, tiles, epi, lds, s)), true)) || ...);
        return r;
    }
};

}  // namespace mmx
