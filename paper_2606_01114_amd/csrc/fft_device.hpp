// Device-side FFT building blocks for gfx950: complex helpers, small radix
// DFTs held in registers, and one Stockham auto-sort stage over lines that
// live in LDS.  Radices 2,3,4,5,7,8,16 cover every 7-smooth length.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmx {

template <typename T> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename T> using cplx = typename cplx_of<T>::type;

template <typename C> __device__ __forceinline__ C cmake(decltype(C().x) a, decltype(C().x) b) { C r; r.x = a; r.y = b; return r; }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) { return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmake<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C().x) s) { return cmake<C>(a.x * s, a.y * s); }
// multiply by DIR*i  (DIR = -1 forward, +1 inverse)
template <int DIR, typename C> __device__ __forceinline__ C cmul_i(C a) {
    return DIR < 0 ? cmake<C>(a.y, -a.x) : cmake<C>(-a.y, a.x);
}
// multiply by cos(t) + DIR*i*sin(t) given c = cos, s = sin
template <int DIR, typename C> __device__ __forceinline__ C crot(C a, decltype(C().x) c, decltype(C().x) s) {
    const decltype(C().x) ss = DIR < 0 ? -s : s;
    return cmake<C>(a.x * c - a.y * ss, a.x * ss + a.y * c);
}

// ---- raw buffer access with hardware range checking ------------------------
// A resource covers `bytes` bytes from a wave-uniform base.  A load at a byte
// offset at or beyond that size returns zero and a store there is dropped, so
// zero padding and ragged line ends need no per-element branches.  Sizes are
// below 2^31 (checked by the host planner), so an offset of 2^31 plus any
// in-range offset is always out of range.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
constexpr uint32_t kBufOff = 0x80000000u;   // an offset that is always out of range
using BufRsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ BufRsrc make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}
template <typename C> __device__ __forceinline__ C buf_load(BufRsrc r, uint32_t off);
template <> __device__ __forceinline__ float2 buf_load<float2>(BufRsrc r, uint32_t off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <> __device__ __forceinline__ double2 buf_load<double2>(BufRsrc r, uint32_t off) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
// non-temporal forms (streaming hint: the line is not kept in the caches
// for reuse), for data a kernel touches once
template <typename C> __device__ __forceinline__ C buf_load_nt(BufRsrc r, uint32_t off);
template <> __device__ __forceinline__ float2 buf_load_nt<float2>(BufRsrc r, uint32_t off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 2));
}
template <> __device__ __forceinline__ double2 buf_load_nt<double2>(BufRsrc r, uint32_t off) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 2));
}
__device__ __forceinline__ void buf_store_nt(BufRsrc r, uint32_t off, float2 v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, off, 0, 2);
}
__device__ __forceinline__ void buf_store_nt(BufRsrc r, uint32_t off, double2 v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), r, off, 0, 2);
}
__device__ __forceinline__ void buf_store(BufRsrc r, uint32_t off, float2 v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(BufRsrc r, uint32_t off, double2 v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), r, off, 0, 0);
}

// ---- small DFTs: X_k = sum_n x_n exp(DIR 2 pi i n k / R), in place -------
template <int R, int DIR, typename C> struct Dft;

template <int DIR, typename C> struct Dft<2, DIR, C> {
    static __device__ __forceinline__ void run(C *v) { C t = v[0]; v[0] = cadd(t, v[1]); v[1] = csub(t, v[1]); }
};

template <int DIR, typename C> struct Dft<4, DIR, C> {
    static __device__ __forceinline__ void run(C *v) {
        C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        C t2 = cadd(v[1], v[3]), t3 = cmul_i<DIR>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2); v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3); v[3] = csub(t1, t3);
    }
};

template <int DIR, typename C> struct Dft<8, DIR, C> {
    static __device__ __forceinline__ void run(C *v) {
        using R = decltype(C().x);
        const R h = R(0.70710678118654752440084436210484904);
        C e[4] = {v[0], v[2], v[4], v[6]};
        C o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, DIR, C>::run(e);
        Dft<4, DIR, C>::run(o);
        o[1] = crot<DIR>(o[1], h, h);
        o[2] = cmul_i<DIR>(o[2]);
        o[3] = crot<DIR>(o[3], -h, h);
#pragma unroll
        for (int k = 0; k < 4; ++k) { v[k] = cadd(e[k], o[k]); v[k + 4] = csub(e[k], o[k]); }
    }
};

template <int DIR, typename C> struct Dft<16, DIR, C> {
    // 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
    static __device__ __forceinline__ void run(C *v) {
        using R = decltype(C().x);
        const R c1 = R(0.92387953251128675612818318939678829), s1 = R(0.38268343236508977172845998403039887);
        const R h = R(0.70710678118654752440084436210484904);
        C y[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            C t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
            Dft<4, DIR, C>::run(t);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = t[k1];
        }
        // twiddles W16^(n2 k1)
        y[1][1] = crot<DIR>(y[1][1], c1, s1);
        y[1][2] = crot<DIR>(y[1][2], h, h);
        y[1][3] = crot<DIR>(y[1][3], s1, c1);
        y[2][1] = crot<DIR>(y[2][1], h, h);
        y[2][2] = cmul_i<DIR>(y[2][2]);
        y[2][3] = crot<DIR>(y[2][3], -h, h);
        y[3][1] = crot<DIR>(y[3][1], s1, c1);
        y[3][2] = crot<DIR>(y[3][2], -h, h);
        y[3][3] = crot<DIR>(y[3][3], -c1, -s1);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            C t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
            Dft<4, DIR, C>::run(t);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
        }
    }
};

// ---- pruned DFTs for zero-padded lines -------------------------------------
// MODE 1: inputs R/2..R-1 are zero and are not read (first stage of a
// transform whose input occupies the lower half of the line); MODE 2: only
// outputs 0..R/2-1 are produced (last stage of a transform of which only the
// lower half is kept).  MODE 0 is the full DFT.
template <int R, int DIR, int MODE, typename C> struct PDft {
    static __device__ __forceinline__ void run(C *v) {
        if constexpr (MODE == 1) {
#pragma unroll
            for (int r = R / 2; r < R; ++r) v[r] = cmake<C>(0, 0);
        }
        Dft<R, DIR, C>::run(v);
    }
};

template <int DIR, typename C> struct PDft<2, DIR, 1, C> {
    static __device__ __forceinline__ void run(C *v) { v[1] = v[0]; }
};
template <int DIR, typename C> struct PDft<2, DIR, 2, C> {
    static __device__ __forceinline__ void run(C *v) { v[0] = cadd(v[0], v[1]); }
};

template <int DIR, typename C> struct PDft<4, DIR, 1, C> {
    static __device__ __forceinline__ void run(C *v) {
        const C a = v[0], b = v[1], t = cmul_i<DIR>(b);
        v[0] = cadd(a, b); v[2] = csub(a, b);
        v[1] = cadd(a, t); v[3] = csub(a, t);
    }
};
template <int DIR, typename C> struct PDft<4, DIR, 2, C> {
    static __device__ __forceinline__ void run(C *v) {
        C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        C t2 = cadd(v[1], v[3]), t3 = cmul_i<DIR>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2); v[1] = cadd(t1, t3);
    }
};

template <int DIR, int MODE, typename C> struct PDft<8, DIR, MODE, C> {
    static __device__ __forceinline__ void run(C *v) {
        if constexpr (MODE == 0) {
            Dft<8, DIR, C>::run(v);
        } else {
            using R = decltype(C().x);
            const R h = R(0.70710678118654752440084436210484904);
            C e[4] = {v[0], v[2], v[4], v[6]};
            C o[4] = {v[1], v[3], v[5], v[7]};
            // inputs 4..7 are the upper halves of the even and odd sub-DFTs
            PDft<4, DIR, MODE == 1 ? 1 : 0, C>::run(e);
            PDft<4, DIR, MODE == 1 ? 1 : 0, C>::run(o);
            o[1] = crot<DIR>(o[1], h, h);
            o[2] = cmul_i<DIR>(o[2]);
            o[3] = crot<DIR>(o[3], -h, h);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                v[k] = cadd(e[k], o[k]);
                if (MODE == 1) v[k + 4] = csub(e[k], o[k]);
            }
        }
    }
};

template <int DIR, int MODE, typename C> struct PDft<16, DIR, MODE, C> {
    // 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.  Inputs 8..15 are n1 = 2, 3
    // (the upper half of every first-layer DFT); outputs 0..7 are k2 = 0, 1
    // (the lower half of every second-layer DFT).
    static __device__ __forceinline__ void run(C *v) {
        if constexpr (MODE == 0) {
            Dft<16, DIR, C>::run(v);
        } else {
            using R = decltype(C().x);
            const R c1 = R(0.92387953251128675612818318939678829), s1 = R(0.38268343236508977172845998403039887);
            const R h = R(0.70710678118654752440084436210484904);
            C y[4][4];
#pragma unroll
            for (int n2 = 0; n2 < 4; ++n2) {
                C t[4] = {v[n2], v[4 + n2], MODE == 1 ? C() : v[8 + n2], MODE == 1 ? C() : v[12 + n2]};
                PDft<4, DIR, MODE == 1 ? 1 : 0, C>::run(t);
#pragma unroll
                for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = t[k1];
            }
            y[1][1] = crot<DIR>(y[1][1], c1, s1);
            y[1][2] = crot<DIR>(y[1][2], h, h);
            y[1][3] = crot<DIR>(y[1][3], s1, c1);
            y[2][1] = crot<DIR>(y[2][1], h, h);
            y[2][2] = cmul_i<DIR>(y[2][2]);
            y[2][3] = crot<DIR>(y[2][3], -h, h);
            y[3][1] = crot<DIR>(y[3][1], s1, c1);
            y[3][2] = crot<DIR>(y[3][2], -h, h);
            y[3][3] = crot<DIR>(y[3][3], -c1, -s1);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) {
                C t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
                PDft<4, DIR, MODE == 2 ? 2 : 0, C>::run(t);
                v[k1] = t[0];
                v[k1 + 4] = t[1];
                if (MODE == 1) { v[k1 + 8] = t[2]; v[k1 + 12] = t[3]; }
            }
        }
    }
};

template <int DIR, typename C> struct Dft<3, DIR, C> {
    static __device__ __forceinline__ void run(C *v) {
        using R = decltype(C().x);
        const R s3 = R(0.86602540378443864676372317075293618);
        C s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        C a = cmake<C>(v[0].x - R(0.5) * s.x, v[0].y - R(0.5) * s.y);
        C b = cscale(cmul_i<DIR>(d), s3);
        v[0] = cadd(v[0], s);
        v[1] = cadd(a, b);
        v[2] = csub(a, b);
    }
};

// odd prime R: X_k = x0 + sum_{n=1}^{(R-1)/2} [ (x_n + x_{R-n}) cos(2pi nk/R)
//                                      + DIR i (x_n - x_{R-n}) sin(2pi nk/R) ]
template <int R_, int DIR, typename C> struct DftOddPrime {
    static __device__ __forceinline__ void run(C *v, const double *cs, const double *sn) {
        using R = decltype(C().x);
        constexpr int H = (R_ - 1) / 2;
        C p[H], q[H];
#pragma unroll
        for (int n = 1; n <= H; ++n) { p[n - 1] = cadd(v[n], v[R_ - n]); q[n - 1] = cmul_i<DIR>(csub(v[n], v[R_ - n])); }
        C out[R_];
        C s0 = v[0];
#pragma unroll
        for (int n = 0; n < H; ++n) s0 = cadd(s0, p[n]);
        out[0] = s0;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            C a = v[0], b = cmake<C>(R(0), R(0));
#pragma unroll
            for (int n = 1; n <= H; ++n) {
                const int idx = (n * k) % R_;
                const R c = R(cs[idx]), s = R(sn[idx]);
                a = cmake<C>(a.x + p[n - 1].x * c, a.y + p[n - 1].y * c);
                b = cmake<C>(b.x + q[n - 1].x * s, b.y + q[n - 1].y * s);
            }
            out[k] = cadd(a, b);
            out[R_ - k] = csub(a, b);
        }
#pragma unroll
        for (int k = 0; k < R_; ++k) v[k] = out[k];
    }
};

template <int DIR, typename C> struct Dft<5, DIR, C> {
    static __device__ __forceinline__ void run(C *v) {
        const double cs[5] = {1.0, 0.30901699437494742410229341718281906, -0.80901699437494742410229341718281906,
                              -0.80901699437494742410229341718281906, 0.30901699437494742410229341718281906};
        const double sn[5] = {0.0, 0.95105651629515357211643933337938214, 0.58778525229247312916870595463907277,
                              -0.58778525229247312916870595463907277, -0.95105651629515357211643933337938214};
        DftOddPrime<5, DIR, C>::run(v, cs, sn);
    }
};

template <int DIR, typename C> struct Dft<7, DIR, C> {
    static __device__ __forceinline__ void run(C *v) {
        const double cs[7] = {1.0, 0.62348980185873353052500488400423981, -0.22252093395631440428890256449679476,
                              -0.90096886790241912623610231950744505, -0.90096886790241912623610231950744505,
                              -0.22252093395631440428890256449679476, 0.62348980185873353052500488400423981};
        const double sn[7] = {0.0, 0.78183148246802980870844452667405775, 0.97492791218182360701813168299393122,
                              0.43388373911755812047576833284835875, -0.43388373911755812047576833284835875,
                              -0.97492791218182360701813168299393122, -0.78183148246802980870844452667405775};
        DftOddPrime<7, DIR, C>::run(v, cs, sn);
    }
};

// ---- one FFT length: factorisation + twiddle-table offsets ---------------
constexpr int kMaxStages = 12;
struct FftDesc {
    int L;                      // transform length
    int nst;                    // number of stages (0 when L == 1)
    int rad[kMaxStages];        // radix of each stage
    int twoff[kMaxStages];      // offset (complex units) of the stage table
};

// Per-thread register budget: each thread holds at most kE complex values per
// stage, i.e. floor(kE / R) butterflies of radix R.
constexpr int kE = 16;

__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t G) {
    // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous run of tiles so neighbouring tiles share that XCD's L2.
    const uint32_t q = G >> 3, r = G & 7u, x = b & 7u;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// One Stockham stage of radix R over `nlines` lines (line l at buf + l*pitch,
// length L, natural order in and out).  Ns = product of earlier radices.
// tw: forward table for this stage, tw[k*(R-1) + r-1] = exp(-2 pi i k r/(Ns R)).
template <typename T, int R, int DIR>
__device__ __forceinline__ void fft_stage(cplx<T> *buf, int nlines, int pitch, int L, int Ns,
                                          const cplx<T> *__restrict__ tw, int tid, int nthr) {
    using C = cplx<T>;
    constexpr int U = kE / R;
    C v[U][R];
    const int nb = L / R;
    const int total = nlines * nb;
    int jj[U], ll[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = tid + u * nthr;
        ll[u] = -1;
        if (b < total) {
            const int line = b / nb, j = b - line * nb;
            ll[u] = line;
            jj[u] = j;
            const C *src = buf + line * pitch;
#pragma unroll
            for (int r = 0; r < R; ++r) v[u][r] = src[j + r * nb];
            const int k = j % Ns;
            if (Ns > 1) {
                const C *t = tw + k * (R - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = t[r - 1];
                    if (DIR > 0) w = cconj(w);
                    v[u][r] = cmul(v[u][r], w);
                }
            }
            Dft<R, DIR, C>::run(v[u]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (ll[u] >= 0) {
            const int j = jj[u];
            const int k = j % Ns;
            const int d = (j / Ns) * Ns * R + k;
            C *dst = buf + ll[u] * pitch;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[d + r * Ns] = v[u][r];
        }
    }
    __syncthreads();
}

// Full transform of `nlines` LDS lines.  Natural order in, natural order out,
// unnormalised.  Ends with a barrier.
template <typename T, int DIR>
__device__ void lds_fft(cplx<T> *buf, int nlines, int pitch, const FftDesc &f, const cplx<T> *__restrict__ tw,
                        int tid, int nthr) {
    int Ns = 1;
    for (int s = 0; s < f.nst; ++s) {
        const int R = f.rad[s];
        const cplx<T> *t = tw + f.twoff[s];
        switch (R) {
        case 16: fft_stage<T, 16, DIR>(buf, nlines, pitch, f.L, Ns, t, tid, nthr); break;
        case 8: fft_stage<T, 8, DIR>(buf, nlines, pitch, f.L, Ns, t, tid, nthr); break;
        case 4: fft_stage<T, 4, DIR>(buf, nlines, pitch, f.L, Ns, t, tid, nthr); break;
        case 2: fft_stage<T, 2, DIR>(buf, nlines, pitch, f.L, Ns, t, tid, nthr); break;
        case 3: fft_stage<T, 3, DIR>(buf, nlines, pitch, f.L, Ns, t, tid, nthr); break;
        case 5: fft_stage<T, 5, DIR>(buf, nlines, pitch, f.L, Ns, t, tid, nthr); break;
        case 7: fft_stage<T, 7, DIR>(buf, nlines, pitch, f.L, Ns, t, tid, nthr); break;
        default: break;
        }
        Ns *= R;
    }
}


// ---- compile-time plans ------------------------------------------------------
// Lengths 2^k, or 2^k q with one odd radix q in {3, 5, 7} as the last
// stage.  Same factorisation as the host planner: the power of two as
// radix-16 stages with an 8/4/2 tail (an exponent = 1 mod 4 ends in 8, 4
// rather than 16, 2), then q.  The first stage is then always even, so a
// line whose upper half is zero skips half of its loads.
namespace ct {
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }
constexpr int odd_part(int L) { return (L >= 2 && L % 2 == 0) ? odd_part(L / 2) : L; }
constexpr int pow2_part(int L) { return L / odd_part(L); }
constexpr int nst2(int L) {
    const int p = ilog2(L), a = p / 4, rem = p % 4;
    return p == 0 ? 0 : p == 1 ? 1 : (rem == 1 && a >= 1) ? a + 1 : a + (rem ? 1 : 0);
}
constexpr int rad2(int L, int s) {
    const int p = ilog2(L), a = p / 4, rem = p % 4;
    return p == 1 ? 2
           : (rem == 1 && a >= 1) ? (s < a - 1 ? 16 : (s == a - 1 ? 8 : 4))
                                  : (s < a ? 16 : (rem == 3 ? 8 : rem == 2 ? 4 : 2));
}
constexpr int nst(int L) { return nst2(pow2_part(L)) + (odd_part(L) > 1 ? 1 : 0); }
constexpr int rad(int L, int s) { return s < nst2(pow2_part(L)) ? rad2(pow2_part(L), s) : odd_part(L); }
constexpr int ns_before(int L, int s) { return s == 0 ? 1 : ns_before(L, s - 1) * rad(L, s - 1); }
constexpr int twoff(int L, int s) { return s == 0 ? 0 : twoff(L, s - 1) + ns_before(L, s - 1) * (rad(L, s - 1) - 1); }
constexpr bool is_pow2(int L) { return L >= 1 && (L & (L - 1)) == 0; }
constexpr bool is_ct_len(int L) {
    return L >= 1 && (odd_part(L) == 1 || odd_part(L) == 3 || odd_part(L) == 5 || odd_part(L) == 7);
}
}  // namespace ct

// One Stockham stage with every size known at compile time.  NLMAX lines at
// most, NT threads; each thread owns U = ceil(NLMAX*L/R / NT) butterflies.
template <typename T, int L, int R, int Ns, int DIR, int NT, int NLMAX>
__device__ __forceinline__ void fft_stage_ct(cplx<T> *buf, int nlines, int pitch, const cplx<T> *__restrict__ tw,
                                             int tid) {
    using C = cplx<T>;
    constexpr int nb = L / R;
    constexpr int U = (NLMAX * nb + NT - 1) / NT;
    const int total = nlines * nb;
    C v[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = tid + u * NT;
        if (b < total) {
            const int line = b / nb, j = b % nb;
            const C *src = buf + line * pitch;
#pragma unroll
            for (int r = 0; r < R; ++r) v[u][r] = src[j + r * nb];
            if (Ns > 1) {
                const int k = j % Ns;
                const C *t = tw + k * (R - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = t[r - 1];
                    if (DIR > 0) w = cconj(w);
                    v[u][r] = cmul(v[u][r], w);
                }
            }
            Dft<R, DIR, C>::run(v[u]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = tid + u * NT;
        if (b < total) {
            const int line = b / nb, j = b % nb;
            const int d = (j / Ns) * Ns * R + (j % Ns);
            C *dst = buf + line * pitch;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[d + r * Ns] = v[u][r];
        }
    }
    __syncthreads();
}

template <typename T, int L, int S, int DIR, int NT, int NLMAX>
__device__ __forceinline__ void fft_ct_from(cplx<T> *buf, int nlines, int pitch, const cplx<T> *__restrict__ tw, int tid) {
    if constexpr (S < ct::nst(L)) {
        constexpr int TWO = ct::twoff(L, S);
        fft_stage_ct<T, L, ct::rad(L, S), ct::ns_before(L, S), DIR, NT, NLMAX>(buf, nlines, pitch, tw + TWO, tid);
        fft_ct_from<T, L, S + 1, DIR, NT, NLMAX>(buf, nlines, pitch, tw, tid);
    }
}

// Full power-of-two transform of up to NLMAX LDS lines (threads >= NT idle).
template <typename T, int L, int DIR, int NT, int NLMAX>
__device__ __forceinline__ void lds_fft_ct(cplx<T> *buf, int nlines, int pitch, const cplx<T> *__restrict__ tw, int tid) {
    fft_ct_from<T, L, 0, DIR, NT, NLMAX>(buf, nlines, pitch, tw, tid < NT ? tid : (1 << 29));
}

// Fast unsigned division by a runtime divisor d >= 1 (n < 2^31):
// q = (umulhi(n, m) + n) >> s with s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1.
struct FastDiv {
    uint32_t d, m, s;
};
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f) {
    return (__umulhi(n, f.m) + n) >> f.s;
}
__host__ __device__ inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    f.s = s;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
    return f;
}

}  // namespace mmx
