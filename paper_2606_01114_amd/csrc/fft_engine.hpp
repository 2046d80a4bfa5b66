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
// Within a line, position p is stored at p + p/16: the radix-R scatter of
// the early Stockham stages then spreads over the LDS banks instead of
// hitting every 16th word.  Power-of-two lines of 32 or more use it; a line
// with an odd radix uses it when every stage's read stride L/R is a multiple
// of 16 (so that the offset form below holds), else it is stored plainly.
constexpr bool swz_strides(int L, int s) {
    return s >= nst(L) ? true : ((L / rad(L, s)) % 16 == 0 && swz_strides(L, s + 1));
}
constexpr bool swz_ok(int L) { return L >= 32 && (is_pow2(L) || swz_strides(L, 0)); }
constexpr int swz(int L, int p) { return swz_ok(L) ? p + (p >> 4) : p; }
constexpr int line_len(int L) { return swz_ok(L) ? L + L / 16 : L; }
// LDS pitch of a line of csz-byte values: the swizzled length plus a shift
// that spreads the NL interleaved lines over the banks.  LDS serves 128 bytes
// (32 four-byte banks) per cycle, i.e. 16 lanes of a 64-bit access or 8 lanes
// of a 128-bit one; the lanes of one such group read or write neighbouring
// lines at the same position, so consecutive lines are shifted by
// (lanes per group / NL) values, or by one when NL covers the group.  Three
// lines (the components of one pencil) take an odd shift that also separates
// the radix-16 scatter of short lines.
constexpr int lds_pitch(int L, int NL, int csz) {
    const int lanes = 128 / csz;
    const int pad = NL == 3 ? (L == 64 ? 7 : L == 128 ? 3 : 11) : (NL >= lanes ? 1 : lanes / (NL < 1 ? 1 : NL));
    return line_len(L) + pad;
}
}  // namespace ct

template <int L> __device__ __forceinline__ int sw(int p) { return ct::swz_ok(L) ? p + (p >> 4) : p; }

// Offset form of the swizzle: sw(a + b) = sw(a) + swc(b) whenever
// (a mod 16) + (b mod 16) < 16.  Every access of a power-of-two Stockham stage
// has that form (a = j or the butterfly's output base, b = a multiple of the
// stride that stays within the 16-block), so per-element addresses become
// compile-time offsets from one per-butterfly base.
template <int L> __device__ __forceinline__ constexpr int swc(int b) { return ct::swz_ok(L) ? b + (b >> 4) : b; }

// LDS slot of position base + r, r < R, of a radix-R output block starting at
// base (a multiple of R): the offset form for R a power of two up to 16, the
// whole swizzle otherwise (a block of odd length can straddle a 16-block)
template <int L, int R> __device__ __forceinline__ int swb(int base, int r) {
    return (R & (R - 1)) == 0 ? sw<L>(base) + swc<L>(r) : sw<L>(base + r);
}

// Twiddle exp(-2 pi i k r / (Ns R)) of a stage in table form TM (see
// eng_stage_la); tt = the stage-ordered table at butterfly class k.
template <int L, int Ns, int R, int TM, class C>
__device__ __forceinline__ C stage_tw(const C *__restrict__ tw, const C *__restrict__ tt, int k, int r) {
    if constexpr (TM == 1) {
        return tw[k * (r * (L / (Ns * R)))];
    } else {
        return tt[r - 1];
    }
}

// One stage.  IN: 0 = from the loader, 1 = from LDS, 2 = from the loader
// with the thread's butterfly round u and input index r as well
// (ld(u, r, line, pos)); OUT: 0 = to the storer,
// 1 = to LDS, 2 = to the storer with the thread's butterfly round u and
// output index r as well (st(u, r, line, pos, C), so that a caller can keep
// the outputs in a register array).  ld(line, pos) -> C; st(line, pos, C).  Butterfly b maps to
// line = b % LA + LA * (b / (LA * NB)), j = (b / LA) % NB: groups of LA lines
// are interleaved (LA = NL: all lines; LA = 3: the components of one cell
// column).  P = LDS pitch of a line.  PR = 1: the line's upper half
// (positions >= L/2, i.e. inputs r >= R/2 of a first stage) is zero and not
// loaded; PR = 2: only the lower half of the output is stored (outputs
// r < R/2 of a last stage).  TM = 0: tw is the stage-ordered twiddle table
// (tw + TWO + k (R-1) + r-1 holds exp(-2 pi i k r / (Ns R))); TM = 1: tw is a
// table of the L roots exp(-2 pi i m / L) (in LDS), entry k r L / (Ns R), the
// same for both radix orders.
template <typename T, int L, bool REV, int S, int DIR, int NT, int NL, int IN, int OUT, int LA, int P, int PR = 0,
          int TM = 0, class Ld, class St>
__device__ __forceinline__ void eng_stage_la(cplx<T> *lds, const cplx<T> *__restrict__ tw, int tid, const Ld &ld, const St &st) {
    using C = cplx<T>;
    constexpr int R = ct::prad(L, REV, S);
    constexpr int Ns = ct::pns(L, REV, S);
    constexpr int NB = L / R;
    constexpr int TOT = NL * NB;
    constexpr int U = (TOT + NT - 1) / NT;
    constexpr int TWO = ct::ptw(L, REV, S);
    constexpr int RI = PR == 1 ? R / 2 : R;   // inputs read
    // outputs written: an odd last radix computes and hands over all of its
    // outputs (the storer's range check drops rows past the kept half)
    constexpr int RO = (PR == 2 && R % 2 == 0) ? R / 2 : R;
    static_assert(PR != 1 || (Ns == 1 && R % 2 == 0), "a zero upper half applies to an even first stage");
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
            for (int r = 0; r < RI; ++r) {
                if constexpr (IN == 1) v[u][r] = lds[sj + swc<L>(r * NB)];
                else if constexpr (IN == 2) v[u][r] = ld(u, r, line, j + r * NB);
                else v[u][r] = ld(line, j + r * NB);
            }
            if (Ns > 1) {
                const int k = j % Ns;
                const C *tt = t + k * (R - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = stage_tw<L, Ns, R, TM>(tw, tt, k, r);
                    if (DIR > 0) w = cconj(w);
                    v[u][r] = cmul(v[u][r], w);
                }
            }
            PDft<R, DIR, PR, C>::run(v[u]);
        }
    }
    if (IN == 1 && OUT == 1) __syncthreads();
    // the offset form of the swizzle holds for the output block d + r Ns when
    // Ns is a multiple of 16 or a power of two with a power-of-two radix;
    // otherwise (the stage after an odd radix in reversed order) each slot
    // is swizzled whole
    constexpr bool WOFF = (Ns % 16 == 0) || (ct::is_pow2(Ns) && ct::is_pow2(R));
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = tid + u * NT;
        if (b < TOT) {
            const int line = b % LA + LA * (b / (LA * NB)), j = (b / LA) % NB;
            const int d = (j / Ns) * Ns * R + (j % Ns);
            const int sd = line * P + sw<L>(d);
#pragma unroll
            for (int r = 0; r < RO; ++r) {
                if constexpr (OUT == 1) lds[WOFF ? sd + swc<L>(r * Ns) : line * P + sw<L>(d + r * Ns)] = v[u][r];
                else if constexpr (OUT == 2) st(u, r, line, d + r * Ns, v[u][r]);
                else st(line, d + r * Ns, v[u][r]);
            }
        }
    }
    if (OUT == 1) __syncthreads();
}

// ---- register-resident transform with half-line LDS exchanges -------------
// Every thread keeps its values in registers from the first stage to the
// last; between two stages the values cross through an LDS buffer that holds
// only half of each line: first the positions in the lower half of the line
// (written by the butterflies that produce them, read by every butterfly of
// the next stage for its inputs r < R/2), then the upper half.  The tile
// needs half the LDS of eng_fft, at the price of two more barriers per
// exchange.  Butterfly b maps to line = b % NL, j = b / NL.
template <int L, bool REV, int S> struct HxStage {
    static constexpr int R = ct::prad(L, REV, S);
    static constexpr int Ns = ct::pns(L, REV, S);
    static constexpr int NB = L / R;
    static constexpr int TWO = ct::ptw(L, REV, S);
};

template <int L, int NL, int CS> constexpr int hx_pitch() { return ct::lds_pitch(L / 2, NL, CS); }

// twiddles and the radix-R DFT of stage S (order REV, table tw) on registers
template <typename T, int L, bool REV, int S, int DIR, int NT, int NL, int PR, int U, int R>
__device__ __forceinline__ void hx_compute(cplx<T> (&v)[U][R], const cplx<T> *__restrict__ tw, int tid) {
    using C = cplx<T>;
    using St = HxStage<L, REV, S>;
    static_assert(St::R == R, "stage shape");
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = tid + u * NT;
        if (b < NL * St::NB) {
            const int j = b / NL;
            if (St::Ns > 1) {
                const C *tt = tw + St::TWO + (j % St::Ns) * (R - 1);
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
}

// Half-line exchange, writer side: the outputs o of stage S (order REV, not
// the last stage) whose block lies in half h.
template <typename T, int L, bool REV, int S, int NT, int NL, int UO, int RO>
__device__ __forceinline__ void hx_put(cplx<T> *lds, const cplx<T> (&o)[UO][RO], int h, int tid) {
    using A = HxStage<L, REV, S>;
    constexpr int PH = hx_pitch<L, NL, (int)sizeof(cplx<T>)>();
    static_assert(A::Ns * A::R <= L / 2, "a stage before the last writes whole blocks of one half");
#pragma unroll
    for (int u = 0; u < UO; ++u) {
        const int b = tid + u * NT;
        if (b < NL * A::NB) {
            const int line = b % NL, j = b / NL;
            if ((j >= A::NB / 2) == (h == 1)) {
                const int d = (j / A::Ns) * A::Ns * A::R + (j % A::Ns) - h * (L / 2);
                const int base = line * PH + sw<L>(d);
#pragma unroll
                for (int r = 0; r < RO; ++r) lds[base + swc<L>(r * A::Ns)] = o[u][r];
            }
        }
    }
}

// Half-line exchange, reader side: the inputs r of half h of stage S
// (order REV) for every butterfly of this thread.
template <typename T, int L, bool REV, int S, int NT, int NL, int UI, int RI>
__device__ __forceinline__ void hx_get(const cplx<T> *lds, cplx<T> (&v)[UI][RI], int h, int tid) {
    using B = HxStage<L, REV, S>;
    constexpr int PH = hx_pitch<L, NL, (int)sizeof(cplx<T>)>();
#pragma unroll
    for (int u = 0; u < UI; ++u) {
        const int b = tid + u * NT;
        if (b < NL * B::NB) {
            const int line = b % NL, j = b / NL;
            const int base = line * PH + sw<L>(j);
#pragma unroll
            for (int r = 0; r < RI / 2; ++r) v[u][h * (RI / 2) + r] = lds[base + swc<L>(r * B::NB)];
        }
    }
}

// outputs o of stage S (not the last) -> inputs v of stage S+1, same order
template <typename T, int L, bool REV, int S, int NT, int NL, int UO, int RO, int UI, int RI>
__device__ __forceinline__ void hx_exchange(cplx<T> *lds, const cplx<T> (&o)[UO][RO], cplx<T> (&v)[UI][RI], int tid) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        hx_put<T, L, REV, S, NT, NL>(lds, o, h, tid);
        __syncthreads();
        hx_get<T, L, REV, S + 1, NT, NL>(lds, v, h, tid);
        __syncthreads();
    }
}

// stages S .. NS-1 on registers v (stage S's inputs); the last stage hands
// its outputs to the storer.  PRL: pruning of the last stage.
template <typename T, int L, int S, int DIR, int NT, int NL, int PRL, int U, int R, class St>
__device__ __forceinline__ void hx_run(cplx<T> *lds, cplx<T> (&v)[U][R], const cplx<T> *__restrict__ tw, int tid,
                                       const St &st) {
    constexpr int NS = ct::nst(L);
    using A = HxStage<L, false, S>;
    hx_compute<T, L, false, S, DIR, NT, NL, S == NS - 1 ? PRL : 0>(v, tw, tid);
    if constexpr (S == NS - 1) {
        constexpr int RO = PRL == 2 ? R / 2 : R;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = tid + u * NT;
            if (b < NL * A::NB) {
                const int line = b % NL, j = b / NL;
                const int d = (j / A::Ns) * A::Ns * R + (j % A::Ns);
#pragma unroll
                for (int r = 0; r < RO; ++r) st(line, d + r * A::Ns, v[u][r]);
            }
        }
    } else {
        using B = HxStage<L, false, S + 1>;
        constexpr int UI = (NL * B::NB + NT - 1) / NT;
        cplx<T> w[UI][B::R];
        hx_exchange<T, L, false, S, NT, NL>(lds, v, w, tid);
        hx_run<T, L, S + 1, DIR, NT, NL, PRL>(lds, w, tw, tid, st);
    }
}

// Full transform: loader -> registers -> (half-line LDS exchanges) -> storer.
// PRUNE as for eng_fft.  Needs two or more stages.
template <typename T, int L, int DIR, int NT, int NL, int PRUNE, class Ld, class St>
__device__ __forceinline__ void eng_fft_hx(cplx<T> *lds, const cplx<T> *__restrict__ tw, int tid, const Ld &ld,
                                           const St &st) {
    static_assert(ct::nst(L) >= 2, "two or more stages");
    using A = HxStage<L, false, 0>;
    constexpr int U = (NL * A::NB + NT - 1) / NT;
    constexpr int RI = (PRUNE & 1) ? A::R / 2 : A::R;
    cplx<T> v[U][A::R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = tid + u * NT;
        if (b < NL * A::NB) {
            const int line = b % NL, j = b / NL;
#pragma unroll
            for (int r = 0; r < RI; ++r) v[u][r] = ld(line, j + r * A::NB);
        }
    }
    // the first stage's pruning is applied in hx_compute through PR below
    using C = cplx<T>;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int b = tid + u * NT;
        if (b < NL * A::NB) PDft<A::R, DIR, (PRUNE & 1) ? 1 : 0, C>::run(v[u]);
    }
    constexpr int NS = ct::nst(L);
    if constexpr (NS == 1) {
        static_assert(NS >= 2, "two or more stages");
    } else {
        using B = HxStage<L, false, 1>;
        constexpr int UI = (NL * B::NB + NT - 1) / NT;
        C w[UI][B::R];
        hx_exchange<T, L, false, 0, NT, NL>(lds, v, w, tid);
        hx_run<T, L, 1, DIR, NT, NL, (PRUNE & 2) ? 2 : 0>(lds, w, tw, tid, st);
    }
}

template <typename T, int L, bool REV, int S, int DIR, int NT, int NL, int IN, int OUT, int PR = 0, int TM = 0,
          class Ld, class St>
__device__ __forceinline__ void eng_stage(cplx<T> *lds, const cplx<T> *__restrict__ tw, int tid, const Ld &ld, const St &st) {
    eng_stage_la<T, L, REV, S, DIR, NT, NL, IN, OUT, NL, ct::lds_pitch(L, NL, (int)sizeof(cplx<T>)), PR, TM>(lds, tw, tid, ld, st);
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

// stages [S, E) all LDS -> LDS (TM as for eng_stage_la)
template <typename T, int L, bool REV, int S, int E, int DIR, int NT, int NL, int TM = 0>
__device__ __forceinline__ void eng_mid(cplx<T> *lds, const cplx<T> *__restrict__ tw, int tid) {
    if constexpr (S < E) {
        auto nold = [](int, int) { return cplx<T>(); };
        auto nost = [](int, int, cplx<T>) {};
        eng_stage<T, L, REV, S, DIR, NT, NL, 1, 1, 0, TM>(lds, tw, tid, nold, nost);
        eng_mid<T, L, REV, S + 1, E, DIR, NT, NL, TM>(lds, tw, tid);
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
