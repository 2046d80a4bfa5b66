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

template <typename T, typename I>
__device__ __forceinline__ T ms_at(const T *Ms, T Ms_s, I cell) { return Ms ? Ms[cell] : Ms_s; }

// Reciprocal and reciprocal square root: the hardware approximations (about
// one ulp) in FP32, correctly rounded division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float rnorm(float n2) { return __builtin_amdgcn_rsqf(n2); }
__device__ __forceinline__ double rnorm(double n2) { return 1.0 / sqrt(n2); }

// maximum that propagates NaN (a non-finite error must not be hidden)
__device__ __forceinline__ double nmax(double a, double b) { return (b > a || b != b) ? b : a; }

// Inputs of one cell's epilogue, loaded before any arithmetic so that the
// loads of several cells can be in flight together.  MSV: Ms is a per-cell
// field (else the scalar).  A neighbour outside the domain is replaced by the
// cell itself (its difference term is exactly zero: the Neumann condition);
// a vacuum neighbour gets weight 0.  LOC: the plan may carry DMI, anisotropy
// or spin-transfer torque (else those terms are compiled out).
// per-thread accumulators of an epilogue: energies (sums 0, 1), the RK
// error (max 0), or the minimiser's dot products (sums 0-2) and torque (max 3)
struct Acc4 {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
};

// stages of the largest Butcher tableau the stage epilogue runs (RKF45: 6)
constexpr int kMaxTabStages = 6;

// I: type of the cell index (int64_t, or int when 3 x cells < 2^31 so that
// every index computation stays in 32 bits; a signed type, whose overflow
// the compiler may assume away, so that it still merges the three component
// loads of a cell into one and folds constant offsets)
template <typename T, typename I = int64_t>
struct CellIn {
    I cell;
    T msi, mi[3], mnb[6][3], msn[6], mn[3], ac[3], gi[3], gnb[6][3], kj[kMaxTabStages - 1][3], mp[3], gp[3];
};

template <typename T, int EPI, bool MSV, bool LOC = true, typename I>
__device__ __forceinline__ void cell_load(const ZInvArgs &a, I cell, int i, int j, int z, CellIn<T, I> &in) {
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const I sx = (I)ny * (I)nz, sy = (I)nz;
    const bool exch = (a.terms & 2u) != 0 || (LOC && a.dmi_kind != 0);   // both read the six neighbours
    const T *Ms = reinterpret_cast<const T *>(a.Ms);
    const T *mfield = reinterpret_cast<const T *>(EPI == EPI_STAGE || EPI == EPI_TAB ? a.ms_in : a.m);
    I nc[6];
    nc[0] = i > 0 ? cell - sx : cell;
    nc[1] = i < nx - 1 ? cell + sx : cell;
    nc[2] = j > 0 ? cell - sy : cell;
    nc[3] = j < ny - 1 ? cell + sy : cell;
    nc[4] = z > 0 ? cell - 1 : cell;
    nc[5] = z < nz - 1 ? cell + 1 : cell;
    in.cell = cell;
    in.msi = MSV ? Ms[cell] : T(a.Ms_scalar);
#pragma unroll
    for (int c = 0; c < 3; ++c) in.mi[c] = mfield[cell * 3 + c];
    if (exch) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
#pragma unroll
            for (int c = 0; c < 3; ++c) in.mnb[q][c] = mfield[nc[q] * 3 + c];
            in.msn[q] = MSV ? Ms[nc[q]] : in.msi;
        }
    }
    if (EPI == EPI_STAGE) {
        const T *mnp = reinterpret_cast<const T *>(a.m_n) + cell * 3;
        const T *accp = reinterpret_cast<const T *>(a.acc) + cell * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) in.mn[c] = mnp[c];
        if (a.stage > 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) in.ac[c] = accp[c];
        }
    }
    if (EPI == EPI_TAB) {
        const T *mnp = reinterpret_cast<const T *>(a.m_n) + cell * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) in.mn[c] = mnp[c];
        const T *K = reinterpret_cast<const T *>(a.K) + cell * 3;
        // compile-time indices keep the earlier stages' derivatives in registers
#pragma unroll
        for (int j = 0; j < kMaxTabStages - 1; ++j) {
            if (j < a.tab_s) {
#pragma unroll
                for (int c = 0; c < 3; ++c) in.kj[j][c] = K[j * a.kstride + c];
            }
        }
    }
    if (EPI == EPI_BB && a.bb_prev) {
        const T *mp = reinterpret_cast<const T *>(a.bb_mprev) + cell * 3;
        const T *gp = reinterpret_cast<const T *>(a.bb_gprev) + cell * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) { in.mp[c] = mp[c]; in.gp[c] = gp[c]; }
    }
    if (EPI == EPI_ADJ) {
        const T *gh = reinterpret_cast<const T *>(a.g_h);
#pragma unroll
        for (int c = 0; c < 3; ++c) in.gi[c] = gh[cell * 3 + c];
        if (exch) {
#pragma unroll
            for (int q = 0; q < 6; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) in.gnb[q][c] = gh[nc[q] * 3 + c];
        }
    }
}

// hd = demag field at the cell (0 if not requested).  Returns in src_next the
// next stage's z-transform source Ms * m_next (EPI_STAGE only).
template <typename T, int EPI, bool MSV, bool LOC = true, typename I>
__device__ __forceinline__ void cell_compute(const ZInvArgs &a, const CellIn<T, I> &in, const T hd[3], Acc4 &acc,
                                             T src_next[3]) {
    const bool exch = (a.terms & 2u) != 0, demag = (a.terms & 1u) != 0;
    const T exp_ = T(a.ex_pref);
    const I cell = in.cell;
    const T msi = in.msi;
    const T *mi = in.mi;
    // ---- exchange field (and DMI, eq. (3), added to it for the dynamics)
    const bool magi = msi > T(0);
    T hex[3] = {T(0), T(0), T(0)};
    T hdm[3] = {T(0), T(0), T(0)};
    T wq[6];
    if (LOC && a.dmi_kind != 0 && magi) {
        // central differences; a missing or vacuum neighbour counts as the cell itself
        T dq[6][3];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const bool ok = !MSV || in.msn[q] > T(0);
#pragma unroll
            for (int c = 0; c < 3; ++c) dq[q][c] = ok ? in.mnb[q][c] - mi[c] : T(0);
        }
        T dm[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) dm[k][c] = (dq[2 * k + 1][c] - dq[2 * k][c]) * T(a.inv_2d[k]);
        const T pd = T(a.dmi_pref) * recip(msi);
        if (a.dmi_kind == 1) {
            // e^DMI = (e_y, -e_x, 0): h = (d_x m_z, d_y m_z, -d_x m_x - d_y m_y)
            hdm[0] = pd * dm[0][2];
            hdm[1] = pd * dm[1][2];
            hdm[2] = -pd * (dm[0][0] + dm[1][1]);
        } else {
            // e^DMI = e_k: h = curl m
            hdm[0] = pd * (dm[1][2] - dm[2][1]);
            hdm[1] = pd * (dm[2][0] - dm[0][2]);
            hdm[2] = pd * (dm[0][1] - dm[1][0]);
        }
    }
    if (LOC && a.ku_pref != 0.0 && magi) {
        // uniaxial anisotropy 2 Ku/(mu0 Ms) (m . u) u, a local term: it goes
        // with the DMI field into every output and right-hand side
        const T ux = T(a.ku_axis[0]), uy = T(a.ku_axis[1]), uz = T(a.ku_axis[2]);
        const T s = T(a.ku_pref) * recip(msi) * (mi[0] * ux + mi[1] * uy + mi[2] * uz);
        hdm[0] += s * ux;
        hdm[1] += s * uy;
        hdm[2] += s * uz;
    }
    if (LOC && a.stt_pref != 0.0 && magi) {
        // Slonczewski torque as a field: beta (eps(m . p) (m x p) + eps' p)
        const T p[3] = {T(a.stt_p[0]), T(a.stt_p[1]), T(a.stt_p[2])};
        const T beta = T(a.stt_pref) * recip(msi);
        const T mp = mi[0] * p[0] + mi[1] * p[1] + mi[2] * p[2];
        const T be = beta * T(a.stt_pl2) * recip(T(a.stt_l2p1) + T(a.stt_l2m1) * mp);
        const T bf = beta * T(a.stt_epsp);
        T mxp[3];
        cross3(mi, p, mxp);
#pragma unroll
        for (int c = 0; c < 3; ++c) hdm[c] += be * mxp[c] + bf * p[c];
    }
    if ((a.terms & 2u) != 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) wq[q] = (MSV && !(in.msn[q] > T(0))) ? T(0) : T(a.inv_d2[q >> 1]);
        T lap[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int q = 0; q < 6; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) lap[c] += (in.mnb[q][c] - mi[c]) * wq[q];
        const T ci = exp_ * recip(msi);
#pragma unroll
        for (int c = 0; c < 3; ++c) hex[c] = magi ? ci * lap[c] : T(0);
    }
    if (EPI == EPI_HEFF) {
        T *ho = reinterpret_cast<T *>(a.h_out) + cell * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) ho[c] = hd[c] + hex[c] + hdm[c] + T(a.hext[c]);
        if (a.epart) {
            acc.v[0] += (double)msi * ((double)mi[0] * hd[0] + (double)mi[1] * hd[1] + (double)mi[2] * hd[2]);
            acc.v[1] += (double)msi * ((double)mi[0] * hex[0] + (double)mi[1] * hex[1] + (double)mi[2] * hex[2]);
        }
    } else if (EPI == EPI_STAGE) {
        T h[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) h[c] = hd[c] + hex[c] + hdm[c] + T(a.hext[c]);
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
        T *acc = reinterpret_cast<T *>(a.acc) + cell * 3;
        const T *mn = in.mn, *ac = in.ac;
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
                const T r = rnorm(nxt[0] * nxt[0] + nxt[1] * nxt[1] + nxt[2] * nxt[2]);
#pragma unroll
                for (int c = 0; c < 3; ++c) nxt[c] *= r;
            }
        }
        T *mo = reinterpret_cast<T *>(a.stage < 3 ? a.ms_out : a.m_out);
        if (mo) {
#pragma unroll
            for (int c = 0; c < 3; ++c) mo[cell * 3 + c] = nxt[c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) src_next[c] = msi * nxt[c];
    } else if (EPI == EPI_TAB) {
        T h[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) h[c] = hd[c] + hex[c] + hdm[c] + T(a.hext[c]);
        T mxh[3], mxmxh[3], f[3];
        cross3(mi, h, mxh);
        cross3(mi, mxh, mxmxh);
        const T gp = T(a.gp), al = T(a.alpha), dt = T(a.dt);
#pragma unroll
        for (int c = 0; c < 3; ++c) f[c] = -gp * (mxh[c] + al * mxmxh[c]);
        const int s = a.tab_s;
        T *K = reinterpret_cast<T *>(a.K) + cell * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) K[s * a.kstride + c] = f[c];
        // sum_j w_j k_j over the earlier stages and this one
        T sa[3], se[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) { sa[c] = T(a.tab_as) * f[c]; se[c] = T(a.tab_es) * f[c]; }
#pragma unroll
        for (int j = 0; j < kMaxTabStages - 1; ++j) {
            if (j < s) {
                const T wa = T(a.tab_a[j]), we = T(a.tab_e[j]);
#pragma unroll
                for (int c = 0; c < 3; ++c) { sa[c] += wa * in.kj[j][c]; se[c] += we * in.kj[j][c]; }
            }
        }
        T nxt[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) nxt[c] = in.mn[c] + dt * sa[c];
        if (!a.tab_last) {
            T *mo = reinterpret_cast<T *>(a.ms_out) + cell * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) mo[c] = nxt[c];
#pragma unroll
            for (int c = 0; c < 3; ++c) src_next[c] = msi * nxt[c];
        } else {
            double e = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) e = nmax(e, (double)fabs(dt * se[c]));
            acc.v[0] = nmax(acc.v[0], e);
            if (a.renorm) {
                const T r = rnorm(nxt[0] * nxt[0] + nxt[1] * nxt[1] + nxt[2] * nxt[2]);
#pragma unroll
                for (int c = 0; c < 3; ++c) nxt[c] *= r;
            }
            T *co = reinterpret_cast<T *>(a.cand) + cell * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) { co[c] = nxt[c]; src_next[c] = T(0); }
        }
    } else if (EPI == EPI_BB) {
        T h[3], mxh[3], g[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) h[c] = hd[c] + hex[c] + hdm[c] + T(a.hext[c]);
        cross3(mi, h, mxh);
        cross3(mi, mxh, g);
        T *go = reinterpret_cast<T *>(a.bb_g) + cell * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) go[c] = g[c];
        const double t2 = (double)mxh[0] * mxh[0] + (double)mxh[1] * mxh[1] + (double)mxh[2] * mxh[2];
        acc.v[3] = nmax(acc.v[3], sqrt(t2));
        if (a.bb_prev) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double s = (double)mi[c] - (double)in.mp[c], y = (double)g[c] - (double)in.gp[c];
                acc.v[0] += s * s;
                acc.v[1] += s * y;
                acc.v[2] += y * y;
            }
        }
    } else {  // EPI_ADJ
        T gm[3] = {T(0), T(0), T(0)};
        T gms = T(0);
        const T *gi = in.gi;
        if (demag) {
#pragma unroll
            for (int c = 0; c < 3; ++c) gm[c] = msi * hd[c];
            gms = mi[0] * hd[0] + mi[1] * hd[1] + mi[2] * hd[2];
        }
        if (exch && magi) {
            const T ci = exp_ * recip(msi);
            T lg[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                // a vacuum neighbour has weight 0 (and would divide by Ms = 0)
                const T cn = wq[q] != T(0) ? exp_ * recip(in.msn[q]) : T(0);
#pragma unroll
                for (int c = 0; c < 3; ++c) lg[c] += (cn * in.gnb[q][c] - ci * gi[c]) * wq[q];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) gm[c] += lg[c];
            gms -= (gi[0] * hex[0] + gi[1] * hex[1] + gi[2] * hex[2]) * recip(msi);
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

// one cell, loads then arithmetic
template <typename T, int EPI>
__device__ __forceinline__ void cell_epilogue(const ZInvArgs &a, int64_t cell, int i, int j, int z, const T hd[3],
                                              Acc4 &acc, T src_next[3]) {
    CellIn<T> in;
    if (a.Ms) {
        cell_load<T, EPI, true>(a, cell, i, j, z, in);
        cell_compute<T, EPI, true>(a, in, hd, acc, src_next);
    } else {
        cell_load<T, EPI, false>(a, cell, i, j, z, in);
        cell_compute<T, EPI, false>(a, in, hd, acc, src_next);
    }
}

// block maximum of one non-negative FP64 value per thread (the RK error);
// a maximum does not depend on the order of the reduction
__device__ __forceinline__ void block_max(double v, double *red, double *out, int tid) {
    __syncthreads();
    for (int off = 32; off > 0; off >>= 1) v = nmax(v, __shfl_down(v, off, 64));
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    if (tid == 0) {
        double m = 0.0;
        const int nw = (blockDim.x + 63) / 64;
        for (int w = 0; w < nw; ++w) m = nmax(m, red[w]);
        out[0] = m;
    }
}

// fixed-order block reduction of the minimiser's three sums and its maximum
__device__ __forceinline__ void block_bb(const Acc4 &acc, double *red, double *out4, int tid) {
    double v0 = acc.v[0], v1 = acc.v[1], v2 = acc.v[2], v3 = acc.v[3];
    __syncthreads();
    for (int off = 32; off > 0; off >>= 1) {
        v0 += __shfl_down(v0, off, 64);
        v1 += __shfl_down(v1, off, 64);
        v2 += __shfl_down(v2, off, 64);
        v3 = nmax(v3, __shfl_down(v3, off, 64));
    }
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) { red[4 * wv] = v0; red[4 * wv + 1] = v1; red[4 * wv + 2] = v2; red[4 * wv + 3] = v3; }
    __syncthreads();
    if (tid == 0) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, mx = 0.0;
        const int nw = (blockDim.x + 63) / 64;
        for (int w = 0; w < nw; ++w) { s0 += red[4 * w]; s1 += red[4 * w + 1]; s2 += red[4 * w + 2]; mx = nmax(mx, red[4 * w + 3]); }
        out4[0] = s0; out4[1] = s1; out4[2] = s2; out4[3] = mx;
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
