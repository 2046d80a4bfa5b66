// Launchers of the compile-time z passes for the folded lengths N = Lz/2
// with one odd radix from 160 on (Lz 320, 384 is in kern_zct_hi.hip, 448,
// 640, 896).
#include "zct_kernels.hpp"

namespace mmx {

template <typename T> using ZctOdd = ZctLengths<T, 160, 192, 224, 320, 448>;

template <typename T>
hipError_t launch_zfwd_ct_odd_b(const ZFwdArgs &a, int src_mode, size_t lds, hipStream_t s) {
    return ZctOdd<T>::fwd(a.g.Lz / 2, a, src_mode, lds, s);
}

template <typename T>
hipError_t launch_zinv_ct_odd_b(const ZInvArgs &a, int epi, size_t lds, hipStream_t s) {
    return ZctOdd<T>::inv(a.g.Lz / 2, a, epi, lds, s);
}

template <typename T>
hipError_t launch_zfwd_ct_b_odd_b(const ZFwdArgs *d, const int2 *map, int tiles, int Lz, int src_mode, size_t lds, hipStream_t s) {
    return ZctOdd<T>::fwd_b(Lz / 2, d, map, tiles, src_mode, lds, s);
}

template <typename T>
hipError_t launch_zinv_ct_b_odd_b(const ZInvArgs *d, const int2 *map, int tiles, int Lz, int epi, size_t lds, hipStream_t s) {
    return ZctOdd<T>::inv_b(Lz / 2, d, map, tiles, epi, lds, s);
}

template hipError_t launch_zfwd_ct_odd_b<float>(const ZFwdArgs &, int, size_t, hipStream_t);
template hipError_t launch_zfwd_ct_odd_b<double>(const ZFwdArgs &, int, size_t, hipStream_t);
template hipError_t launch_zinv_ct_odd_b<float>(const ZInvArgs &, int, size_t, hipStream_t);
template hipError_t launch_zinv_ct_odd_b<double>(const ZInvArgs &, int, size_t, hipStream_t);
template hipError_t launch_zfwd_ct_b_odd_b<float>(const ZFwdArgs *, const int2 *, int, int, int, size_t, hipStream_t);
template hipError_t launch_zfwd_ct_b_odd_b<double>(const ZFwdArgs *, const int2 *, int, int, int, size_t, hipStream_t);
template hipError_t launch_zinv_ct_b_odd_b<float>(const ZInvArgs *, const int2 *, int, int, int, size_t, hipStream_t);
template hipError_t launch_zinv_ct_b_odd_b<double>(const ZInvArgs *, const int2 *, int, int, int, size_t, hipStream_t);

}  // namespace mmx
