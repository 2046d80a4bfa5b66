// Field evaluations without the demag term (h_eff of the exchange stencil and
// the local fields alone) as a streaming stencil.  The cells of one x plane
// are contiguous (index q = y nz + z), so a workgroup owns a contiguous range
// of q and marches along x: the previous, current and next plane of its own
// cells stay in registers (the x neighbours), and the current plane with one y
// row of halo on each side goes through LDS (the y and z neighbours).  Each
// value of m is read from HBM about once.  The per-cell arithmetic is the z
// pass epilogue's (cell_compute), so both paths give identical fields.
#include <algorithm>

#include "passes.hpp"
#include "kernels.hpp"
#include "zepi.hpp"

namespace mmx {

namespace {
constexpr int kStQB = 1024;             // plane cells per workgroup
constexpr int kStMaxNz = 512;           // halo of one y row on each side
// threads per workgroup: two own cells per thread, one in FP64 without the
// local terms (the register budget of the planes in flight at 1024 threads)
template <typename T, bool LOC> constexpr int st_threads() { return sizeof(T) == 8 && !LOC ? 1024 : 512; }
}  // namespace

template <typename T, bool MSV, bool LOC>
__global__ void __launch_bounds__((st_threads<T, LOC>())) k_stencil_heff(const ZInvArgs a, int cx, int nqb) {
    constexpr int kStNT = st_threads<T, LOC>();
    constexpr int kStQ = kStQB / kStNT;           // own cells per thread and plane
    constexpr int kStHQ = 2 * kStMaxNz / kStNT;   // halo cells per thread
    extern __shared__ __align__(16) unsigned char smem[];
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int plane = ny * nz;                       // < 2^31 (host check)
    const uint32_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int qb = (int)(t % (uint32_t)nqb), xc = (int)(t / (uint32_t)nqb);
    const int q0 = qb * kStQB;
    const int x0 = xc * cx, x1 = min(nx, x0 + cx);
    const int span = kStQB + 2 * nz;                 // LDS cells: [q0 - nz, q0 + QB + nz)
    T *sm = reinterpret_cast<T *>(smem);             // [span][3]
    T *ss = sm + 3 * span;                           // [span] (per-cell Ms)
    const T *m = reinterpret_cast<const T *>(a.m);
    const T *Ms = reinterpret_cast<const T *>(a.Ms);
    const int tid = threadIdx.x;
    const T zero[3] = {T(0), T(0), T(0)};
    Acc4 acc;
    if (x0 >= x1) {
        if (a.epart) block_energy(acc.v[0], acc.v[1], reinterpret_cast<double *>(smem), a.epart + 2 * (int64_t)blockIdx.x, tid);
        return;
    }
    auto load = [&](int x, int q, T (&v)[3], T &s) {
        const int64_t c = (int64_t)x * plane + q;
#pragma unroll
        for (int k = 0; k < 3; ++k) v[k] = m[c * 3 + k];
        s = MSV ? Ms[c] : T(a.Ms_scalar);
    };
    // own cells: q = q0 + tid + k NT; planes x-1, x, x+1 and the prefetched x+2
    T mp[kStQ][3], mc[kStQ][3], mn[kStQ][3], mf[kStQ][3];
    T sp[kStQ], sc[kStQ], sn[kStQ], sf[kStQ];
    // halo cells of the next plane: e = tid + k NT < 2 nz, q = q0 - nz + e
    // (e < nz) or q0 + QB + e - nz
    T hv[kStHQ][3], hs[kStHQ];
    auto halo_q = [&](int e) { return e < nz ? q0 - nz + e : q0 + kStQB + (e - nz); };
    auto load_halo = [&](int x) {
#pragma unroll
        for (int k = 0; k < kStHQ; ++k) {
            const int e = tid + k * kStNT;
            const int q = halo_q(e);
            if (e < 2 * nz && q >= 0 && q < plane) load(x, q, hv[k], hs[k]);
        }
    };
#pragma unroll
    for (int k = 0; k < kStQ; ++k) {
        const int q = q0 + tid + k * kStNT;
        if (q < plane) {
            load(x0, q, mc[k], sc[k]);
            if (x0 > 0) load(x0 - 1, q, mp[k], sp[k]);
            if (x0 + 1 < nx) load(x0 + 1, q, mn[k], sn[k]);
        }
    }
    load_halo(x0);
    for (int x = x0; x < x1; ++x) {
        // prefetch plane x+2 of the own cells
        if (x + 2 < nx && x + 1 < x1) {
#pragma unroll
            for (int k = 0; k < kStQ; ++k) {
                const int q = q0 + tid + k * kStNT;
                if (q < plane) load(x + 2, q, mf[k], sf[k]);
            }
        }
        // current plane into LDS: own cells and halo
#pragma unroll
        for (int k = 0; k < kStQ; ++k) {
            const int q = q0 + tid + k * kStNT;
            if (q < plane) {
                const int e = nz + tid + k * kStNT;
#pragma unroll
                for (int c = 0; c < 3; ++c) sm[e * 3 + c] = mc[k][c];
                if (MSV) ss[e] = sc[k];
            }
        }
#pragma unroll
        for (int k = 0; k < kStHQ; ++k) {
            const int e = tid + k * kStNT;
            const int q = halo_q(e);
            if (e < 2 * nz && q >= 0 && q < plane) {
                const int el = e < nz ? e : e + kStQB;
#pragma unroll
                for (int c = 0; c < 3; ++c) sm[el * 3 + c] = hv[k][c];
                if (MSV) ss[el] = hs[k];
            }
        }
        __syncthreads();
        if (x + 1 < x1) load_halo(x + 1);
#pragma unroll
        for (int k = 0; k < kStQ; ++k) {
            const int q = q0 + tid + k * kStNT;
            if (q < plane) {
                const int e = nz + tid + k * kStNT;
                const int y = (int)fdiv((uint32_t)q, a.g.dnz), z = q - y * nz;
                CellIn<T> in;
                in.cell = (int64_t)x * plane + q;
                in.msi = sc[k];
                const int en[4] = {y > 0 ? e - nz : e, y < ny - 1 ? e + nz : e, z > 0 ? e - 1 : e, z < nz - 1 ? e + 1 : e};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    in.mi[c] = mc[k][c];
                    in.mnb[0][c] = x > 0 ? mp[k][c] : mc[k][c];
                    in.mnb[1][c] = x < nx - 1 ? mn[k][c] : mc[k][c];
                }
                in.msn[0] = x > 0 ? sp[k] : sc[k];
                in.msn[1] = x < nx - 1 ? sn[k] : sc[k];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) in.mnb[2 + u][c] = sm[en[u] * 3 + c];
                    in.msn[2 + u] = MSV ? ss[en[u]] : sc[k];
                }
                T srcn[3];
                cell_compute<T, EPI_HEFF, MSV, LOC>(a, in, zero, acc, srcn);
            }
        }
        __syncthreads();
        // rotate the planes
#pragma unroll
        for (int k = 0; k < kStQ; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) { mp[k][c] = mc[k][c]; mc[k][c] = mn[k][c]; mn[k][c] = mf[k][c]; }
            sp[k] = sc[k]; sc[k] = sn[k]; sn[k] = sf[k];
        }
    }
    if (a.epart) block_energy(acc.v[0], acc.v[1], reinterpret_cast<double *>(smem), a.epart + 2 * (int64_t)blockIdx.x, tid);
}

// Launch shape: x chunks of cx planes so that the grid has about 2048
// workgroups and no more than max_blocks (the energy partial slots).
// Returns 0 when the grid does not fit the kernel (nz > 512, a plane of 2^31
// cells or more, or more plane blocks than slots).
int stencil_shape(int nx, int ny, int nz, int max_blocks, int *cx, int *nqb, int *blocks) {
    const int64_t plane = (int64_t)ny * nz;
    if (nz > kStMaxNz || plane >= (int64_t(1) << 31)) return 0;
    const int q = (int)((plane + kStQB - 1) / kStQB);
    if (q > max_blocks) return 0;
    int nxc = (int)std::min<int64_t>(nx, std::max<int64_t>(1, (2048 + q - 1) / q));
    nxc = std::min(nxc, std::max(1, max_blocks / q));
    int c = (nx + nxc - 1) / nxc;
    nxc = (nx + c - 1) / c;
    *cx = c;
    *nqb = q;
    *blocks = q * nxc;
    return 1;
}

size_t stencil_lds(int nz, size_t rsz) {
    const size_t span = (size_t)kStQB + 2 * (size_t)nz;
    return std::max<size_t>(span * 4 * rsz, 2 * 8 * (1024 / 64));   // fields, or the energy reduction
}

template <typename T>
hipError_t launch_stencil_heff(const ZInvArgs &a, int cx, int nqb, int blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    const size_t lds = stencil_lds(a.g.nz, sizeof(T));
    const bool msv = a.Ms != nullptr;
    const bool loc = a.dmi_kind != 0 || a.ku_pref != 0.0 || a.stt_pref != 0.0;
    constexpr int nl = st_threads<T, true>(), np = st_threads<T, false>();
    if (msv && loc) hipLaunchKernelGGL((k_stencil_heff<T, true, true>), dim3(blocks), dim3(nl), lds, s, a, cx, nqb);
    else if (msv) hipLaunchKernelGGL((k_stencil_heff<T, true, false>), dim3(blocks), dim3(np), lds, s, a, cx, nqb);
    else if (loc) hipLaunchKernelGGL((k_stencil_heff<T, false, true>), dim3(blocks), dim3(nl), lds, s, a, cx, nqb);
    else hipLaunchKernelGGL((k_stencil_heff<T, false, false>), dim3(blocks), dim3(np), lds, s, a, cx, nqb);
    return hipGetLastError();
}

template hipError_t launch_stencil_heff<float>(const ZInvArgs &, int, int, int, hipStream_t);
template hipError_t launch_stencil_heff<double>(const ZInvArgs &, int, int, int, hipStream_t);

}  // namespace mmx
