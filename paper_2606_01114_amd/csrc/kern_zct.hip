// Launchers of the compile-time z passes.  The folded lengths N = Lz/2 up to
// 32 are instantiated here, the longer ones in kern_zct_hi.hip (the two
// files compile in parallel).
#include "zct_kernels.hpp"

namespace mmx {

int zct_cols(int Lz) {
    if (Lz < 2 || Lz > 2048) return 0;
    if (Lz & (Lz - 1)) {
        switch (Lz) {
        case 96: case 160: case 192: case 224: case 320: case 384: case 448: case 640: case 768: case 896: break;
        default: return 0;
        }
    }
    return zcols(Lz / 2);
}

size_t zct_lds(int Lz, size_t csz) {
    const int N = Lz / 2;
    return std::max<size_t>((size_t)3 * zcols(N) * zpitch(N) * csz, 512);
}

int zinv_ct_tiles(int nx, int ny, int Lz, int ygrp) { return ztile_count(nx, ny, zcols(Lz / 2), ygrp); }

template <typename T> using ZctLo = ZctLengths<T, 1, 2, 4, 8, 16, 32>;

template <typename T>
hipError_t launch_zfwd_ct(const ZFwdArgs &a, int src_mode, hipStream_t s) {
    const int N = a.g.Lz / 2;
    const size_t lds = zct_lds(a.g.Lz, sizeof(cplx<T>));
    const hipError_t r = ZctLo<T>::fwd(N, a, src_mode, lds, s);
    return r == hipErrorInvalidValue ? launch_zfwd_ct_hi<T>(a, src_mode, lds, s) : r;
}

template <typename T>
hipError_t launch_zinv_ct(const ZInvArgs &a, int epi, hipStream_t s) {
    const int N = a.g.Lz / 2;
    const size_t lds = zct_lds(a.g.Lz, sizeof(cplx<T>));
    const hipError_t r = ZctLo<T>::inv(N, a, epi, lds, s);
    return r == hipErrorInvalidValue ? launch_zinv_ct_hi<T>(a, epi, lds, s) : r;
}

template <typename T>
hipError_t launch_zfwd_ct_b(const ZFwdArgs *d, const int2 *map, int tiles, int Lz, int src_mode, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    const size_t lds = zct_lds(Lz, sizeof(cplx<T>));
    const hipError_t r = ZctLo<T>::fwd_b(Lz / 2, d, map, tiles, src_mode, lds, s);
    return r == hipErrorInvalidValue ? launch_zfwd_ct_b_hi<T>(d, map, tiles, Lz, src_mode, lds, s) : r;
}

template <typename T>
hipError_t launch_zinv_ct_b(const ZInvArgs *d, const int2 *map, int tiles, int Lz, int epi, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    const size_t lds = zct_lds(Lz, sizeof(cplx<T>));
    const hipError_t r = ZctLo<T>::inv_b(Lz / 2, d, map, tiles, epi, lds, s);
    return r == hipErrorInvalidValue ? launch_zinv_ct_b_hi<T>(d, map, tiles, Lz, epi, lds, s) : r;
}

template hipError_t launch_zfwd_ct_b<float>(const ZFwdArgs *, const int2 *, int, int, int, hipStream_t);
template hipError_t launch_zfwd_ct_b<double>(const ZFwdArgs *, const int2 *, int, int, int, hipStream_t);
template hipError_t launch_zinv_ct_b<float>(const ZInvArgs *, const int2 *, int, int, int, hipStream_t);
template hipError_t launch_zinv_ct_b<double>(const ZInvArgs *, const int2 *, int, int, int, hipStream_t);
template hipError_t launch_zfwd_ct<float>(const ZFwdArgs &, int, hipStream_t);
template hipError_t launch_zfwd_ct<double>(const ZFwdArgs &, int, hipStream_t);
template hipError_t launch_zinv_ct<float>(const ZInvArgs &, int, hipStream_t);
template hipError_t launch_zinv_ct<double>(const ZInvArgs &, int, hipStream_t);

}  // namespace mmx
