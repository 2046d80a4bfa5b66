// Launchers of the compile-time z passes for the power-of-two folded lengths
// N = Lz/2 of 64 and more and for 384 (kern_zct.hip has the shorter ones and
// calls these; the other odd-radix lengths are in kern_zct_odd_a/b.hip).
#include "zct_kernels.hpp"

namespace mmx {

template <typename T> using ZctHi = ZctLengths<T, 64, 128, 256, 384, 512, 1024>;

template <typename T>
hipError_t launch_zfwd_ct_hi(const ZFwdArgs &a, int src_mode, size_t lds, hipStream_t s) {
    hipError_t r = ZctHi<T>::fwd(a.g.Lz / 2, a, src_mode, lds, s);
    if (r == hipErrorInvalidValue) r = launch_zfwd_ct_odd_a<T>(a, src_mode, lds, s);
    return r == hipErrorInvalidValue ? launch_zfwd_ct_odd_b<T>(a, src_mode, lds, s) : r;
}

template <typename T>
hipError_t launch_zinv_ct_hi(const ZInvArgs &a, int epi, size_t lds, hipStream_t s) {
    hipError_t r = ZctHi<T>::inv(a.g.Lz / 2, a, epi, lds, s);
    if (r == hipErrorInvalidValue) r = launch_zinv_ct_odd_a<T>(a, epi, lds, s);
    return r == hipErrorInvalidValue ? launch_zinv_ct_odd_b<T>(a, epi, lds, s) : r;
}

template <typename T>
hipError_t launch_zfwd_ct_b_hi(const ZFwdArgs *d, const int2 *map, int tiles, int Lz, int src_mode, size_t lds, hipStream_t s) {
    hipError_t r = ZctHi<T>::fwd_b(Lz / 2, d, map, tiles, src_mode, lds, s);
    if (r == hipErrorInvalidValue) r = launch_zfwd_ct_b_odd_a<T>(d, map, tiles, Lz, src_mode, lds, s);
    return r == hipErrorInvalidValue ? launch_zfwd_ct_b_odd_b<T>(d, map, tiles, Lz, src_mode, lds, s) : r;
}

template <typename T>
hipError_t launch_zinv_ct_b_hi(const ZInvArgs *d, const int2 *map, int tiles, int Lz, int epi, size_t lds, hipStream_t s) {
    hipError_t r = ZctHi<T>::inv_b(Lz / 2, d, map, tiles, epi, lds, s);
    if (r == hipErrorInvalidValue) r = launch_zinv_ct_b_odd_a<T>(d, map, tiles, Lz, epi, lds, s);
    return r == hipErrorInvalidValue ? launch_zinv_ct_b_odd_b<T>(d, map, tiles, Lz, epi, lds, s) : r;
}

template hipError_t launch_zfwd_ct_hi<float>(const ZFwdArgs &, int, size_t, hipStream_t);
template hipError_t launch_zfwd_ct_hi<double>(const ZFwdArgs &, int, size_t, hipStream_t);
template hipError_t launch_zinv_ct_hi<float>(const ZInvArgs &, int, size_t, hipStream_t);
template hipError_t launch_zinv_ct_hi<double>(const ZInvArgs &, int, size_t, hipStream_t);
template hipError_t launch_zfwd_ct_b_hi<float>(const ZFwdArgs *, const int2 *, int, int, int, size_t, hipStream_t);
template hipError_t launch_zfwd_ct_b_hi<double>(const ZFwdArgs *, const int2 *, int, int, int, size_t, hipStream_t);
template hipError_t launch_zinv_ct_b_hi<float>(const ZInvArgs *, const int2 *, int, int, int, size_t, hipStream_t);
template hipError_t launch_zinv_ct_b_hi<double>(const ZInvArgs *, const int2 *, int, int, int, size_t, hipStream_t);

}  // namespace mmx
