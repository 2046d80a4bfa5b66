// Launch wrappers of the HIP kernels (host-callable).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "passes.hpp"

namespace mmx {

template <typename T>
hipError_t launch_line_pass(const LinePass *d_descs, const int2 *d_map, int tiles, int nthr, size_t lds_bytes, int dir,
                            bool sym, hipStream_t s);
template <typename T>
hipError_t launch_fused_y(const FusedPass *d_descs, const int2 *d_map, int tiles, int nthr, size_t lds_bytes,
                          hipStream_t s);
// power-of-two specialisations; line_ct_shape / fused_ct_threads report
// whether one exists for a length (and its tile width / thread count)
int line_ct_shape(int L, size_t csz, int variant, int *W, int *NT);
int fused_ct_threads(int L, size_t csz);
size_t line_ct_lds(int L, int W, size_t csz);
size_t line_hx_lds(int L, int W, size_t csz);
// register-resident fused y pass: threads (0 = no such kernel) and LDS bytes
int fused_hx_threads(int L);
size_t fused_hx_lds(int L, size_t csz);
template <typename T> hipError_t launch_fused_hx(const FusedPass &a, hipStream_t s);
size_t fused_ct_lds(int L, size_t csz);
// persistent fused y pass with the next pencil's loads in flight (variants 2..4)
int fused_pf_available(int L, int var);
template <typename T> hipError_t launch_fused_pf(const FusedPass &a, int var, hipStream_t s);
// half != 0 launches the half-LDS variant (k_line_hx)
template <typename T> hipError_t launch_line_ct(const LinePass &a, int tiles, int W, int dir, hipStream_t s, int half = 0);
template <typename T> hipError_t launch_line_wide(const LinePass &a, int tiles, int W, int dir, hipStream_t s);
template <typename T>
hipError_t launch_line_wide_b(const LinePass *d, const int2 *map, int tiles, int L, int W, int dir, hipStream_t s);
template <typename T> hipError_t launch_fused_ct(const FusedPass &a, hipStream_t s);
template <typename T> hipError_t launch_zfwd(const ZFwdArgs &a, int src_mode, size_t lds_bytes, hipStream_t s);
template <typename T> hipError_t launch_zinv(const ZInvArgs &a, int epi, size_t lds_bytes, hipStream_t s);
template <typename T>
hipError_t launch_zfwd_batch(const ZFwdArgs *d, const int2 *map, int tiles, int nthr, int src_mode, size_t lds_bytes,
                             hipStream_t s);
template <typename T>
hipError_t launch_zinv_batch(const ZInvArgs *d, const int2 *map, int tiles, int nthr, int epi, size_t lds_bytes,
                             hipStream_t s);
hipError_t launch_copy16(const void *src, void *dst, int64_t n16, hipStream_t s);
// compile-time z passes (power-of-two Lz in [2, 2048] and Lz = 96, 160, 192,
// 224, 320, 384, 448, 640, 768, 896); zct_cols returns the
// cell columns per tile (0 if no specialisation), zct_lds the LDS bytes
int zct_cols(int Lz);
// tiles of the compile-time z-inverse pass (ZGeom::ygrp order)
int zinv_ct_tiles(int nx, int ny, int Lz, int ygrp);
size_t zct_lds(int Lz, size_t csz);
template <typename T> hipError_t launch_zfwd_ct(const ZFwdArgs &a, int src_mode, hipStream_t s);
template <typename T> hipError_t launch_zinv_ct(const ZInvArgs &a, int epi, hipStream_t s);
// the longer folded lengths (kern_zct_hi.hip) and those with an odd radix
// (kern_zct_odd_a/b.hip), called in turn by the four launchers above and
// below; hipErrorInvalidValue for a length they do not have
template <typename T> hipError_t launch_zfwd_ct_hi(const ZFwdArgs &a, int src_mode, size_t lds, hipStream_t s);
template <typename T> hipError_t launch_zinv_ct_hi(const ZInvArgs &a, int epi, size_t lds, hipStream_t s);
template <typename T>
hipError_t launch_zfwd_ct_b_hi(const ZFwdArgs *d, const int2 *map, int tiles, int Lz, int src_mode, size_t lds, hipStream_t s);
template <typename T>
hipError_t launch_zinv_ct_b_hi(const ZInvArgs *d, const int2 *map, int tiles, int Lz, int epi, size_t lds, hipStream_t s);
template <typename T> hipError_t launch_zfwd_ct_odd_a(const ZFwdArgs &a, int src_mode, size_t lds, hipStream_t s);
template <typename T> hipError_t launch_zinv_ct_odd_a(const ZInvArgs &a, int epi, size_t lds, hipStream_t s);
template <typename T>
hipError_t launch_zfwd_ct_b_odd_a(const ZFwdArgs *d, const int2 *map, int tiles, int Lz, int src_mode, size_t lds, hipStream_t s);
template <typename T>
hipError_t launch_zinv_ct_b_odd_a(const ZInvArgs *d, const int2 *map, int tiles, int Lz, int epi, size_t lds, hipStream_t s);
template <typename T> hipError_t launch_zfwd_ct_odd_b(const ZFwdArgs &a, int src_mode, size_t lds, hipStream_t s);
template <typename T> hipError_t launch_zinv_ct_odd_b(const ZInvArgs &a, int epi, size_t lds, hipStream_t s);
template <typename T>
hipError_t launch_zfwd_ct_b_odd_b(const ZFwdArgs *d, const int2 *map, int tiles, int Lz, int src_mode, size_t lds, hipStream_t s);
template <typename T>
hipError_t launch_zinv_ct_b_odd_b(const ZInvArgs *d, const int2 *map, int tiles, int Lz, int epi, size_t lds, hipStream_t s);
template <typename T> hipError_t launch_fused_ct_b(const FusedPass *d, const int2 *map, int tiles, int L, hipStream_t s);
// grouped launches in any variant (x: 0..3 as mm_plan_info; y: 0..2)
template <typename T>
hipError_t launch_line_var_b(const LinePass *d, const int2 *map, int tiles, int L, int W, int dir, int var,
                             hipStream_t s);
template <typename T>
hipError_t launch_fused_var_b(const FusedPass *d, const int2 *map, int tiles, int L, int var, hipStream_t s);
template <typename T>
hipError_t launch_zfwd_ct_b(const ZFwdArgs *d, const int2 *map, int tiles, int Lz, int src_mode, hipStream_t s);
template <typename T>
hipError_t launch_zinv_ct_b(const ZInvArgs *d, const int2 *map, int tiles, int Lz, int epi, hipStream_t s);
hipError_t launch_energy_reduce(const double *part, int nblk, double *out, hipStream_t s);
// h_eff without the demag term as a streaming stencil (kern_stencil.hip)
int stencil_shape(int nx, int ny, int nz, int max_blocks, int *cx, int *nqb, int *blocks);
size_t stencil_lds(int nz, size_t rsz);
template <typename T>
hipError_t launch_stencil_heff(const ZInvArgs &a, int cx, int nqb, int blocks, hipStream_t s);
hipError_t launch_max_reduce(const double *part, int nblk, double *out, hipStream_t s);
hipError_t launch_bb_reduce(const double *part, int nblk, double *out4, hipStream_t s);
template <typename T> hipError_t launch_bb_update(T *m, const T *g, T *mprev, double tau, int64_t ncell, hipStream_t s);
hipError_t launch_tensor_octant(double *out, int nx, int ny, int nz, double dx, double dy, double dz, double P,
                                hipStream_t s);
template <typename T>
hipError_t launch_tensor_finalize(const double *in, T *out, int hx, int hy, int hz, double inv_ltot, hipStream_t s);
template <typename T> hipError_t launch_tensor_export(const T *in, double *out, int hx, int hy, int hz, hipStream_t s);
template <typename T>
hipError_t launch_adj_unorm(const T *g, const T *u, T *ub, T *gsum, int renorm, int64_t ncell, hipStream_t s);
template <typename T>
hipError_t launch_adj_combine(const T *ym, const T *gmh, const T *ub, T *gsum, T *kb, double w, double coef, int64_t n,
                              hipStream_t s);

// device address of this device's fixed scratch array (kern_scratch.hip)
hipError_t noalloc_scratch(int device, void **out);

template <typename T> hipError_t launch_scale_copy(const T *in, T *out, double s, int64_t n, hipStream_t st);

}  // namespace mmx
