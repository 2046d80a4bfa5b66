// Descriptors shared by the host planner and the pass kernels.  Every pass is
// a launch over tiles; a descriptor holds one geometry's view of the pass, and
// a batched launch maps each tile to (descriptor, local tile).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "fft_device.hpp"

namespace mmx {

// Strided line transform: lines along one axis, batch columns contiguous.
//   element (outer o, row r, column c) sits at  base + o*outer_stride + r*row + c
// (complex units for complex data, real units in the symmetric mode).
struct LinePass {
    const void *in;
    void *out;
    const void *tw;            // twiddle table of f
    int64_t in_row, out_row, in_outer, out_outer;
    int inner, outer;          // columns per outer index, number of outer indices
    int n_in, n_out;           // rows read (rest zero), rows written
    int W, tiles_inner;        // columns per tile, tiles per outer index
    int pitch, nthr;           // LDS line pitch (complex), threads used
    int sym_axis;              // symmetric real transform: parity axis (0,1,2)
    int pad_;
    FftDesc f;
};

// Fused pass along y: forward FFT, 3x3 spectral product with the demag
// tensor, inverse FFT; in place on S2 laid out [kz][kx][y][component], so the
// three components of one (kz, kx) pencil are one contiguous block.
struct FusedPass {
    void *data;
    const void *tensor;        // [kz][kx'][ky'][6], pre-scaled, kx' <= Lx/2, ky' <= Ly/2
    const void *tw;
    const void *roots;         // exp(-2 pi i m / Ly), m < Ly (compile-time Ly)
    const void *twh;           // stage-ordered tables of length Ly/2, forward then reversed radix order
                               // (compile-time Ly with a half-spectrum kernel; else null)
    int n;                     // rows present along y (ny)
    int Lx, Ly, hz, hxp, hyp;  // hxp = Lx/2+1, hyp = Ly/2+1
    int npos;                  // pencils = hz*Lx
    int W, tiles, pitch, nthr; // pencils per tile, tiles, LDS pitch, threads
    FftDesc f;                 // length Ly
};

// Field constants for the z passes and the fused epilogue.
struct ZGeom {
    int nx, ny, nz, Lz, hz;
    int P, tiles, pitch, nthr; // positions (x,y columns) per tile, linear tiles, ...
    // z-inverse tiles of the compile-time kernels: 0 = linear runs of P
    // positions; > 0 = P positions of one x row, ordered in groups of ygrp
    // y-blocks with x fastest within a group (see ztile)
    int ygrp;
    FftDesc f;                 // length Lz
    const void *tw;
    const void *twh;           // power-of-two Lz: table of length Lz/2, then exp(-2 pi i k/Lz), k <= Lz/2
    void *S1;                  // [kz][pos][c], pos = x*ny + y
    FastDiv dnz, dny;          // division by nz, ny
};

enum SrcMode { SRC_MS_M = 0, SRC_RAW = 1, SRC_ADJPRE = 2 };

// Arguments of the z-forward (R2C) pass.
struct ZFwdArgs {
    ZGeom g;
    const void *src;           // (nx,ny,nz,3)
    const void *Ms;            // per-cell or null
    double Ms_scalar;
    // SRC_ADJPRE: y = VJP of the LLG right-hand side at (s, h) for cotangent kb
    const void *s, *h, *kb;
    void *ym, *yh;
    double gp, alpha;          // gamma/(1+alpha^2), alpha
};

enum EpiMode { EPI_HEFF = 0, EPI_STAGE = 1, EPI_ADJ = 2, EPI_TAB = 3, EPI_BB = 4 };

// Arguments of the z-inverse (C2R) pass and its epilogue.
struct ZInvArgs {
    ZGeom g;
    unsigned terms;            // MM_DEMAG | MM_EXCHANGE bits
    const void *Ms; double Ms_scalar;
    double ex_pref;            // 2A/mu0
    double inv_d2[3];
    int dmi_kind;              // 0 none, 1 interfacial, 2 bulk (eq. (3))
    double dmi_pref;           // 2D/mu0
    double inv_2d[3];          // 1/(2 d_k): central differences
    double ku_pref;            // 2 Ku/mu0 (uniaxial anisotropy; 0 = none)
    double ku_axis[3];         // unit easy axis
    // Slonczewski spin-transfer torque as a field: beta_i = stt_pref / Ms_i,
    // eps(x) = stt_pl2 / (stt_l2p1 + stt_l2m1 x), h = beta (eps (m x p) + stt_epsp p)
    double stt_pref;           // hbar j / (mu0 e d); 0 = none
    double stt_pl2, stt_l2p1, stt_l2m1, stt_epsp;
    double stt_p[3];           // unit polarisation
    double hext[3];
    // heff
    const void *m; void *h_out; double *epart;  // epart: per-block (E_d, E_ex) partials or null
    // stage
    int stage;                 // 0..3
    int next_r2c;              // write the next stage's z spectrum into S1
    int renorm;
    double dt, gp, alpha;
    const void *ms_in, *m_n; void *acc, *ms_out, *m_out, *h_rec, *u_rec;
    // adjoint
    const void *g_h; void *g_m, *g_Ms; int acc_gMs;
    // explicit Runge-Kutta stage from a Butcher tableau (EPI_TAB; uses dt,
    // gp, alpha, renorm, ms_in, m_n, ms_out, next_r2c above): stage tab_s
    // writes its derivative k_s to K + tab_s * kstride; before the last stage
    // the next stage input m_n + dt sum_j tab_a[j] k_j goes to ms_out; the
    // last stage writes the solution m_n + dt sum_j tab_a[j] k_j (renormalised
    // when renorm) to cand and the per-block max over cells and components of
    // |dt sum_j tab_e[j] k_j| to epart[2 blk]
    int i32;                   // every cell and S1 index fits in a signed 32-bit int (compile-time z kernels)
    int tab_s, tab_last;
    double tab_a[8], tab_e[8];   // weights of the earlier stages j < tab_s
    double tab_as, tab_es;       // weights of this stage's own derivative
    void *K; int64_t kstride; void *cand;
    // energy minimisation (EPI_BB; uses m, hext): writes g = m x (m x h) to
    // bb_g and per block (sum s.s, sum s.y, sum y.y, max |m x h|) to
    // bb_part[4 blk], with s = m - bb_mprev, y = g - bb_gprev when bb_prev
    void *bb_g; const void *bb_mprev, *bb_gprev; int bb_prev; double *bb_part;
};

}  // namespace mmx
