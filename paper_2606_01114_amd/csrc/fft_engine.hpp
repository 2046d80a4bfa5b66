// Register-staged Stockham engine for power-of-two lengths known at compile
// time.  A tile holds NL independent lines of length L.  The first stage
// reads its inputs straight from global memory through a loader and the last
// stage hands its outputs straight to a storer, so a transform of S stages
// needs S-1 LDS exchanges instead of S+1.  Butterflies are numbered
// b = line + NL * j (line fastest) so neighbouring threads touch neighbouring
// columns of a row-major tile.
#pragma once
#include "fft_device.hpp"

namespace mmx {
namespace ct {
// radix of stage s in forward (REV = false) or reversed order
constexpr int prad(int L, bool rev, int s) { return rev ? rad(L, nst(L) - 1 - s) : rad(L, s); }
constexpr int pns(int L, bool rev, int s) { return s == 0 ? 1 : pns(L, rev, s - 1) * prad(L, rev, s - 1); }
constexpr int ptw(int L, bool rev, int s) { return s == 0 ? 0 : ptw(L, rev, s - 1) + pns(L, rev, s - 1) * (prad(L, rev, s - 1) - 1); }
// Within a line, position p is stored at p + p/16 (lines of 32 or more):
// the radix-R scatter of the early Stockham stages then spreads over the
// LDS banks instead of hitting every 16th word.
constexpr int swz(int L, int p) { return L >= 32 ? p + (p >> 4) : p; }
constexpr int line_len(int L) { return L >= 32 ? L + L / 16 : L; }
// LDS pitch of a line (swizzled length plus a shift that spreads the NL
// interleaved lines over the banks)
constexpr int lds_pitch(int L, int NL) {
    return line_len(L) + (NL >= 32 ? 1 : (NL == 3 ? 11 : 32 / (NL < 1 ? 1 : NL)));
}
}  // namespace ct

template <int L> __device__ __forceinline__ int sw(int p) { return L >= 32 ? p + (p >> 4) : p; }

// Offset form of the swizzle: sw(a + b) = sw(a) + swc(b) whenever
// (a mod 16) + (b mod 16) < 16.  Every access of a power-of-two Stockham stage
// has that form (a = j or the butterfly's output base, b = a multiple of the
// stride that stays within the 16-block), so per-element addresses become
// compile-time offsets from one per-butterfly base.
template <int L> __device__ __forceinline__ constexpr int swc(int b) { return L >= 32 ? b + (b >> 4) : b; }

// One stage.  IN: 0 = from the loader, 1 = from LDS; OUT: 0 = to the storer,
// 1 = to LDS.  ld(line, pos) -> C; st(line, pos, C).  Butterfly b maps to
// line = b % LA + LA * (b / (LA * NB)), j = (b / LA) % NB: groups of LA lines
// are interleaved (LA = NL: all lines; LA = 3: the components of one cell
// column).  P = LDS pitch of a line.  PR = 1: the line's upper half
// (positions >= L/2, i.e. inputs r >= R/2 of a first stage) is zero and not
// loaded; PR = 2: only the lower half of the output is stored (outputs
// r < R/2 of a last stage).
template <typename T, int L, bool REV, int S, int DIR, int NT, int NL, int IN, int OUT, int LA, int P, int PR = 0,
          class Ld, class St>
__device__ __forceinline__ void eng_stage_la(cplx<T> *lds, const cplx<T> *__restrict__ tw, int tid, const Ld &ld, const St &st) {
    using C = cplx<T>;
    constexpr int R = ct::prad(L, REV, S);
    constexpr int Ns = ct::pns(L, REV, S);
    constexpr int NB = L / R;
    constexpr int TOT = NL * NB;
    constexpr int U = (TOT + NT - 1) / NT;
    constexpr int TWO = ct::ptw(L, REV, S);
    constexpr int RI = PR == 1 ? R / 2 : R;   // inputs read
    constexpr int RO = PR == 2 ? R / 2 : R;   // outputs written
    static_assert(PR != 1 || Ns == 1, "a zero upper half applies to a first stage");
    static_assert(PR != 2 || Ns * R == L, "a half output applies to a last stage");
    const C *t = tw + TWO;
    C v[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = tid + u * NT;
        if (b < TOT) {
            const int line = b % LA + LA * (b / (LA * NB)), j = (b / LA) % NB;
            const int sj = line * P + sw<L>(j);
#pragma unroll
            for (int r = 0; r < RI; ++r) v[u][r] = IN ? lds[sj + swc<L>(r * NB)] : ld(line, j + r * NB);
            if (Ns > 1) {
                const C *tt = t + (j % Ns) * (R - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = tt[r - 1];
                    if (DIR > 0) w = cconj(w);
                    v[u][r] = cmul(v[u][r], w);
                }
            }
            PDft<R, DIR, PR, C>::run(v[u]);
        }
    }
    if (IN && OUT) __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = tid + u * NT;
        if (b < TOT) {
            const int line = b % LA + LA * (b / (LA * NB)), j = (b / LA) % NB;
            const int d = (j / Ns) * Ns * R + (j % Ns);
            const int sd = line * P + sw<L>(d);
#pragma unroll
            for (int r = 0; r < RO; ++r) {
                if (OUT) lds[sd + swc<L>(r * Ns)] = v[u][r];
                else st(line, d + r * Ns, v[u][r]);
            }
        }
    }
    if (OUT) __syncthreads();
}

// The first stage split in two, so that a tile's first-stage inputs can be
// loaded (eng_load0) while the previous tile is still being transformed, and
// transformed later (eng_stage0_regs: registers -> LDS, ends with a barrier).
template <typename T, int L, int NT, int NL>
struct Stage0Regs {
    static constexpr int R = ct::prad(L, false, 0);
    static constexpr int NB = L / R;
    static constexpr int TOT = NL * NB;
    static constexpr int U = (TOT + NT - 1) / NT;
    cplx<T> v[U][R];
};

template <typename T, int L, int NT, int NL, int PR, class Ld>
__device__ __forceinline__ void eng_load0(Stage0Regs<T, L, NT, NL> &s, int tid, const Ld &ld) {
    using S = Stage0Regs<T, L, NT, NL>;
    constexpr int RI = PR == 1 ? S::R / 2 : S::R;
#pragma unroll
    for (int u = 0; u < S::U; ++u) {
        const int b = tid + u * NT;
        if (b < S::TOT) {
            const int line = b % NL, j = b / NL;
#pragma unroll
            for (int r = 0; r < RI; ++r) s.v[u][r] = ld(line, j + r * S::NB);
        }
    }
}

template <typename T, int L, int DIR, int NT, int NL, int PR>
__device__ __forceinline__ void eng_stage0_regs(cplx<T> *lds, Stage0Regs<T, L, NT, NL> &s, int tid) {
    using S = Stage0Regs<T, L, NT, NL>;
    constexpr int P = ct::lds_pitch(L, NL);
    static_assert(ct::nst(L) >= 2, "the split first stage needs a later stage");
#pragma unroll
    for (int u = 0; u < S::U; ++u) {
        const int b = tid + u * NT;
        if (b < S::TOT) {
            const int line = b % NL, j = b / NL;
            PDft<S::R, DIR, PR, cplx<T>>::run(s.v[u]);
            const int sd = line * P + sw<L>(j * S::R);
#pragma unroll
            for (int r = 0; r < S::R; ++r) lds[sd + swc<L>(r)] = s.v[u][r];
        }
    }
    __syncthreads();
}

template <typename T, int L, bool REV, int S, int DIR, int NT, int NL, int IN, int OUT, int PR = 0, class Ld, class St>
__device__ __forceinline__ void eng_stage(cplx<T> *lds, const cplx<T> *__restrict__ tw, int tid, const Ld &ld, const St &st) {
    eng_stage_la<T, L, REV, S, DIR, NT, NL, IN, OUT, NL, ct::lds_pitch(L, NL), PR>(lds, tw, tid, ld, st);
}

// stages [S, E) LDS -> LDS with interleave LA and pitch P
template <typename T, int L, bool REV, int S, int E, int DIR, int NT, int NL, int LA, int P>
__device__ __forceinline__ void eng_mid_la(cplx<T> *lds, const cplx<T> *__restrict__ tw, int tid) {
    if constexpr (S < E) {
        auto nold = [](int, int) { return cplx<T>(); };
        auto nost = [](int, int, cplx<T>) {};
        eng_stage_la<T, L, REV, S, DIR, NT, NL, 1, 1, LA, P>(lds, tw, tid, nold, nost);
        eng_mid_la<T, L, REV, S + 1, E, DIR, NT, NL, LA, P>(lds, tw, tid);
    }
}

// General transform: stage 0 from the loader (IN0 = 0) or LDS (IN0 = 1), the
// last stage to the storer (OUTL = 0) or LDS (OUTL = 1).  With IN0 = 1 the
// caller must have synchronised after filling LDS; with OUTL = 1 the call
// ends with a barrier.  PRUNE as for eng_fft (two or more stages only; the
// skipped upper half is neither read nor written in LDS either).
template <typename T, int L, int DIR, int NT, int NL, int LA, int P, int IN0, int OUTL, int PRUNE = 0, class Ld, class St>
__device__ __forceinline__ void eng_fft_la(cplx<T> *lds, const cplx<T> *__restrict__ tw, int tid, const Ld &ld, const St &st) {
    constexpr int NS = ct::nst(L);
    if constexpr (NS == 0) {
        if constexpr (IN0 == 0) {
            for (int line = tid; line < NL; line += NT) {
                if constexpr (OUTL) lds[line * P] = ld(line, 0);
                else st(line, 0, ld(line, 0));
            }
        } else if constexpr (OUTL == 0) {
            for (int line = tid; line < NL; line += NT) st(line, 0, lds[line * P]);
        }
        if constexpr (OUTL) __syncthreads();
    } else if constexpr (NS == 1) {
        eng_stage_la<T, L, false, 0, DIR, NT, NL, IN0, OUTL, LA, P>(lds, tw, tid, ld, st);
    } else {
        auto nold = [](int, int) { return cplx<T>(); };
        auto nost = [](int, int, cplx<T>) {};
        constexpr int P0 = (PRUNE & 1) ? 1 : 0, PL = (PRUNE & 2) ? 2 : 0;
        eng_stage_la<T, L, false, 0, DIR, NT, NL, IN0, 1, LA, P, P0>(lds, tw, tid, ld, nost);
        eng_mid_la<T, L, false, 1, NS - 1, DIR, NT, NL, LA, P>(lds, tw, tid);
        eng_stage_la<T, L, false, NS - 1, DIR, NT, NL, 1, OUTL, LA, P, PL>(lds, tw, tid, nold, st);
    }
}

// stages [S, E) all LDS -> LDS
template <typename T, int L, bool REV, int S, int E, int DIR, int NT, int NL>
__device__ __forceinline__ void eng_mid(cplx<T> *lds, const cplx<T> *__restrict__ tw, int tid) {
    if constexpr (S < E) {
        auto nold = [](int, int) { return cplx<T>(); };
        auto nost = [](int, int, cplx<T>) {};
        eng_stage<T, L, REV, S, DIR, NT, NL, 1, 1>(lds, tw, tid, nold, nost);
        eng_mid<T, L, REV, S + 1, E, DIR, NT, NL>(lds, tw, tid);
    }
}

// Full transform: loader -> [LDS stages] -> storer.  PRUNE bit 0: the input
// occupies the lower half of each line (upper half zero, not loaded); bit 1:
// only the lower half of each output line is stored.  Transforms of two or
// more stages only.
template <typename T, int L, bool REV, int DIR, int NT, int NL, int PRUNE = 0, class Ld, class St>
__device__ __forceinline__ void eng_fft(cplx<T> *lds, const cplx<T> *__restrict__ tw, int tid, const Ld &ld, const St &st) {
    constexpr int NS = ct::nst(L);
    if constexpr (NS == 0) {
        // length 1: identity
        for (int line = tid; line < NL; line += NT) st(line, 0, ld(line, 0));
    } else if constexpr (NS == 1) {
        eng_stage<T, L, REV, 0, DIR, NT, NL, 0, 0>(lds, tw, tid, ld, st);
    } else {
        eng_stage<T, L, REV, 0, DIR, NT, NL, 0, 1, (PRUNE & 1) ? 1 : 0>(lds, tw, tid, ld, st);
        eng_mid<T, L, REV, 1, NS - 1, DIR, NT, NL>(lds, tw, tid);
        eng_stage<T, L, REV, NS - 1, DIR, NT, NL, 1, 0, (PRUNE & 2) ? 2 : 0>(lds, tw, tid, ld, st);
    }
}

}  // namespace mmx
