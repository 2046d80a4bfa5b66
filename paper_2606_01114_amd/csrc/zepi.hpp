// Per-cell epilogue of the inverse z pass: the 6-point exchange stencil
// (Neumann boundaries, vacuum cells excluded), then either the h_eff output
// (with FP64 energy partial sums), the LLG right-hand side with one classic
// RK4 stage update, or the adjoint of h_eff.  Shared by the runtime-planned
// and the compile-time z kernels.
#pragma once
#include "passes.hpp"

namespace mmx {

template <typename T>
__device__ __forceinline__ void cross3(const T a[3], const T b[3], T o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

template <typename T>
__device__ __forceinline__ T ms_at(const T *Ms, T Ms_s, int64_t cell) { return Ms ? Ms[cell] : Ms_s; }

// The cell's own inputs, fetched ahead of the z transform so their latency
// overlaps it: m (stage input or h_eff input), m_n, the RK4 accumulator, Ms.
template <typename T>
struct OwnCell {
    T mi[3], mn[3], acc[3], ms;
};

template <typename T, int EPI>
__device__ __forceinline__ void load_own(const ZInvArgs &a, int64_t cell, OwnCell<T> &o) {
    const T *mfield = reinterpret_cast<const T *>(EPI == EPI_STAGE ? a.ms_in : a.m);
    const T *Ms = reinterpret_cast<const T *>(a.Ms);
    o.ms = Ms ? Ms[cell] : T(a.Ms_scalar);
#pragma unroll
    for (int c = 0; c < 3; ++c) o.mi[c] = mfield[cell * 3 + c];
    if (EPI == EPI_STAGE) {
        const T *mn = reinterpret_cast<const T *>(a.m_n);
#pragma unroll
        for (int c = 0; c < 3; ++c) o.mn[c] = mn[cell * 3 + c];
        if (a.stage > 0) {
            const T *acc = reinterpret_cast<const T *>(a.acc);
#pragma unroll
            for (int c = 0; c < 3; ++c) o.acc[c] = acc[cell * 3 + c];
        }
    }
}

// cell (i, j, z) with flat index `cell`; hd = demag field there (0 if not
// requested).  Returns in src_next the next stage's z-transform source
// Ms * m_next (EPI_STAGE with next_r2c only).  `pre` (nullable) holds the
// cell's own inputs already loaded.
template <typename T, int EPI>
__device__ __forceinline__ void cell_epilogue(const ZInvArgs &a, int64_t cell, int i, int j, int z, const T hd[3],
                                              double &ed, double &ex, T src_next[3], const OwnCell<T> *pre = nullptr) {
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int64_t sx = (int64_t)ny * nz, sy = nz;
    const bool exch = (a.terms & 2u) != 0, demag = (a.terms & 1u) != 0;
    const T *Ms = reinterpret_cast<const T *>(a.Ms);
    const T Ms_s = T(a.Ms_scalar);
    const T exp_ = T(a.ex_pref);
    const T *mfield = reinterpret_cast<const T *>(EPI == EPI_STAGE ? a.ms_in : a.m);
    const T msi = pre ? pre->ms : ms_at(Ms, Ms_s, cell);
    const bool magi = msi > T(0);
    T mi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) mi[c] = pre ? pre->mi[c] : mfield[cell * 3 + c];
    const int64_t noff[6] = {-sx, sx, -sy, sy, -1, 1};
    const bool nin[6] = {i > 0, i < nx - 1, j > 0, j < ny - 1, z > 0, z < nz - 1};
    T hex[3] = {T(0), T(0), T(0)};
    if (exch && magi) {
        T lap[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            if (!nin[q]) continue;
            const int64_t nc = cell + noff[q];
            if (!(ms_at(Ms, Ms_s, nc) > T(0))) continue;
            const T w = T(a.inv_d2[q >> 1]);
#pragma unroll
            for (int c = 0; c < 3; ++c) lap[c] += (mfield[nc * 3 + c] - mi[c]) * w;
        }
        const T ci = exp_ / msi;
#pragma unroll
        for (int c = 0; c < 3; ++c) hex[c] = ci * lap[c];
    }
    if (EPI == EPI_HEFF) {
        T *ho = reinterpret_cast<T *>(a.h_out) + cell * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) ho[c] = hd[c] + hex[c] + T(a.hext[c]);
        if (a.epart) {
            ed += (double)msi * ((double)mi[0] * hd[0] + (double)mi[1] * hd[1] + (double)mi[2] * hd[2]);
            ex += (double)msi * ((double)mi[0] * hex[0] + (double)mi[1] * hex[1] + (double)mi[2] * hex[2]);
        }
    } else if (EPI == EPI_STAGE) {
        T h[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) h[c] = hd[c] + hex[c] + T(a.hext[c]);
        if (a.h_rec) {
            T *hr = reinterpret_cast<T *>(a.h_rec) + cell * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) hr[c] = h[c];
        }
        T mxh[3], mxmxh[3], f[3];
        cross3(mi, h, mxh);
        cross3(mi, mxh, mxmxh);
        const T gp = T(a.gp), al = T(a.alpha), dt = T(a.dt);
#pragma unroll
        for (int c = 0; c < 3; ++c) f[c] = -gp * (mxh[c] + al * mxmxh[c]);
        const T *mnp = reinterpret_cast<const T *>(a.m_n) + cell * 3;
        T *acc = reinterpret_cast<T *>(a.acc) + cell * 3;
        T mn[3], ac[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) mn[c] = pre ? pre->mn[c] : mnp[c];
        if (a.stage > 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) ac[c] = pre ? pre->acc[c] : acc[c];
        }
        T nxt[3];
        if (a.stage == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) { acc[c] = f[c]; nxt[c] = mn[c] + T(0.5) * dt * f[c]; }
        } else if (a.stage == 1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) { acc[c] = ac[c] + T(2) * f[c]; nxt[c] = mn[c] + T(0.5) * dt * f[c]; }
        } else if (a.stage == 2) {
#pragma unroll
            for (int c = 0; c < 3; ++c) { acc[c] = ac[c] + T(2) * f[c]; nxt[c] = mn[c] + dt * f[c]; }
        } else {
            const T w = dt / T(6);
#pragma unroll
            for (int c = 0; c < 3; ++c) nxt[c] = mn[c] + w * (ac[c] + f[c]);
            if (a.u_rec) {
                T *ur = reinterpret_cast<T *>(a.u_rec) + cell * 3;
#pragma unroll
                for (int c = 0; c < 3; ++c) ur[c] = nxt[c];
            }
            if (a.renorm) {
                const T nn = sqrt(nxt[0] * nxt[0] + nxt[1] * nxt[1] + nxt[2] * nxt[2]);
#pragma unroll
                for (int c = 0; c < 3; ++c) nxt[c] = nxt[c] / nn;
            }
        }
        if (a.stage < 3) {
            T *mo = reinterpret_cast<T *>(a.ms_out) + cell * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) mo[c] = nxt[c];
        } else if (a.m_out) {
            T *mo = reinterpret_cast<T *>(a.m_out) + cell * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) mo[c] = nxt[c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) src_next[c] = msi * nxt[c];
    } else {  // EPI_ADJ
        const T *gh = reinterpret_cast<const T *>(a.g_h);
        T gi[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) gi[c] = gh[cell * 3 + c];
        T gm[3] = {T(0), T(0), T(0)};
        T gms = T(0);
        if (demag) {
#pragma unroll
            for (int c = 0; c < 3; ++c) gm[c] = msi * hd[c];
            gms = mi[0] * hd[0] + mi[1] * hd[1] + mi[2] * hd[2];
        }
        if (exch && magi) {
            const T ci = exp_ / msi;
            T lg[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                if (!nin[q]) continue;
                const int64_t nc = cell + noff[q];
                const T msn = ms_at(Ms, Ms_s, nc);
                if (!(msn > T(0))) continue;
                const T cn = exp_ / msn;
                const T w = T(a.inv_d2[q >> 1]);
#pragma unroll
                for (int c = 0; c < 3; ++c) lg[c] += (cn * gh[nc * 3 + c] - ci * gi[c]) * w;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) gm[c] += lg[c];
            gms -= (gi[0] * hex[0] + gi[1] * hex[1] + gi[2] * hex[2]) / msi;
        }
        T *go = reinterpret_cast<T *>(a.g_m) + cell * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) go[c] = gm[c];
        if (a.g_Ms) {
            T *gM = reinterpret_cast<T *>(a.g_Ms) + cell;
            gM[0] = a.acc_gMs ? gM[0] + gms : gms;
        }
    }
}

// fixed-order block reduction of the two FP64 energy partial sums
__device__ __forceinline__ void block_energy(double ed, double ex, double *red, double *out2, int tid) {
    __syncthreads();
    for (int off = 32; off > 0; off >>= 1) {
        ed += __shfl_down(ed, off, 64);
        ex += __shfl_down(ex, off, 64);
    }
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) { red[2 * wv] = ed; red[2 * wv + 1] = ex; }
    __syncthreads();
    if (tid == 0) {
        double s0 = 0.0, s1 = 0.0;
        const int nw = (blockDim.x + 63) / 64;
        for (int w = 0; w < nw; ++w) { s0 += red[2 * w]; s1 += red[2 * w + 1]; }
        out2[0] = s0;
        out2[1] = s1;
    }
}

}  // namespace mmx
