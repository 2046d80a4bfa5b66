// Host side of the library: argument validation, plans (FFT factorisation,
// twiddle tables, tile choice, workspace), the C ABI declared in mmx.h, and
// HIP-graph capture of the LLG step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mmx.h"
#include "kernels.hpp"
#include "passes.hpp"

using namespace mmx;

namespace {

thread_local std::string g_last = "";

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last = buf;
    return code;
}

#define HIPCK(expr)                                                                             \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(MM_EHIP, "%s: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

const double kMu0 = 4e-7 * M_PI;
const double kHbar = 1.054571817e-34;     // J s (CODATA 2018)
const double kECharge = 1.602176634e-19;  // C (exact in the SI since 2019)
const size_t kLdsMax = 160 * 1024;        // LDS per workgroup on gfx950
const size_t kLdsTarget = 80 * 1024;      // default budget: two workgroups per CU

bool is_7smooth(int64_t v) {
    if (v < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (v % p == 0) v /= p;
    return v == 1;
}

int64_t pow2_L(int64_t n) {
    if (n == 1) return 1;
    int64_t L = 1;
    while (L < 2 * n - 1) L <<= 1;
    return L;
}

int64_t default_L(int64_t n) {
    if (n == 1) return 1;
    if (is_7smooth(n)) return 2 * n;
    int64_t L = 2 * n - 1;
    while (!is_7smooth(L)) ++L;
    return L;
}

// Lengths an axis has compile-time kernels for: powers of two (x and y up to
// 4096, an FP64 y pencil and z up to 2048) and q * 2^k with one odd radix q
// (x and y: 96, 160, 192, 224, 320, 384, 448, 640, 768, 896, 1280, 1536,
// 1792; z the same up to 896).
bool ct_len_ok(int64_t L, int axis, int precision) {
    const int64_t lim = axis == 2 ? 2048 : (axis == 1 && precision == MM_F64 ? 2048 : 4096);
    if ((L & (L - 1)) == 0) return L <= lim;
    switch (L) {
    case 96: case 160: case 192: case 224: case 320: case 384: case 448:
    case 640: case 768: case 896: return true;
    case 1280: case 1536: case 1792: return axis != 2;
    default: return false;
    }
}

// the smallest compile-time length >= 2n-1 (a power of two past the table)
int64_t ct_L(int64_t n, int axis, int precision) {
    if (n == 1) return 1;
    int64_t best = 0;
    for (int64_t q = 1; q <= 4096; q <<= 1)
        for (int64_t m : {1, 3, 5, 7}) {
            const int64_t L = q * m;
            if (L >= 2 * n - 1 && ct_len_ok(L, axis, precision) && (!best || L < best)) best = L;
        }
    return best ? best : pow2_L(n);
}

// Automatic padding of one axis: the shortest compile-time length when it is
// at most 1.75 times the 7-smooth length, else the 7-smooth length.  The
// compile-time kernels move the extra padded bytes faster than the
// runtime-planned mixed-radix kernels move the smaller problem (FP64 demag of
// an N^3 cube with powers of two only: N = 350, 1024^3 16.0 ms against 700^3
// 26.3 ms; N = 160, 512^3 1.69 ms against 320^3 2.22 ms; but N = 260, 1024^3
// 12.6 ms against 525^3 11.0 ms).
int64_t auto_L(int64_t n, int axis, int precision) {
    const int64_t s = default_L(n), q = ct_L(n, axis, precision);
    return (ct_len_ok(q, axis, precision) && 4 * q <= 7 * s) ? q : s;
}

std::vector<int> factorize(int L) {
    std::vector<int> r;
    int p2 = 0;
    while (L % 2 == 0) { L /= 2; ++p2; }
    if (p2 == 1) r.push_back(2);
    else if (p2 > 1) {
        int a = p2 / 4, rem = p2 % 4;
        if (rem == 1 && a >= 1) { a -= 1; r.insert(r.end(), a, 16); r.push_back(8); r.push_back(4); }
        else {
            r.insert(r.end(), a, 16);
            if (rem == 3) r.push_back(8);
            else if (rem == 2) r.push_back(4);
            else if (rem == 1) r.push_back(2);
        }
    }
    for (int p : {3, 5, 7})
        while (L % p == 0) { L /= p; r.push_back(p); }
    return r;
}

// a radix order written as "4,5,5,7"
std::vector<int> parse_order(const std::string &t) {
    std::vector<int> o;
    size_t i = 0;
    while (i < t.size()) {
        o.push_back(atoi(t.c_str() + i));
        const size_t c = t.find(',', i);
        if (c == std::string::npos) break;
        i = c + 1;
    }
    return o;
}

struct HostFft {
    FftDesc d;
    std::vector<long double> tw;   // interleaved re, im; forward sign
};

// radix order `order` (a permutation of factorize(L)); empty: the default
HostFft make_fft(int L, bool rev = false, const std::vector<int> &order = {}) {
    HostFft h;
    std::memset(&h.d, 0, sizeof h.d);
    h.d.L = L;
    std::vector<int> rad = order.empty() ? factorize(L) : order;
    if (rev) std::reverse(rad.begin(), rad.end());
    h.d.nst = (int)rad.size();
    int Ns = 1, off = 0;
    for (size_t s = 0; s < rad.size(); ++s) {
        const int R = rad[s];
        h.d.rad[s] = R;
        h.d.twoff[s] = off;
        for (int k = 0; k < Ns; ++k)
            for (int r = 1; r < R; ++r) {
                const long long num = ((long long)k * r) % ((long long)Ns * R);
                const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)num / (long double)(Ns * R);
                h.tw.push_back(cosl(ang));
                h.tw.push_back(sinl(ang));
            }
        off += Ns * (R - 1);
        Ns *= R;
    }
    return h;
}

// threads needed so that every stage fits the per-thread register budget
int fft_threads(const FftDesc &d, int nlines, int min_work) {
    int need = 64;
    for (int s = 0; s < d.nst; ++s) {
        const int R = d.rad[s];
        const int U = kE / R;
        const long long bf = (long long)nlines * (d.L / R);
        need = std::max<long long>(need, (bf + U - 1) / U);
    }
    need = std::max(need, std::min(min_work, 256));
    need = (need + 63) / 64 * 64;
    return need;
}

int pitch_of(int L) { return (L % 2 == 0) ? L + 1 : L; }

}  // namespace

struct mm_plan {
    int prec = MM_F32;
    size_t rsz = 4;
    int64_t n[3] = {0, 0, 0};
    double d[3] = {0, 0, 0};
    int64_t L[3] = {0, 0, 0};
    int hx = 0, hy = 0, hz = 0;
    double P = 16.0;
    int dmi_kind = 0;          // 0 none, 1 interfacial, 2 bulk
    double dmi_D = 0.0;        // J/m^2
    double ku = 0.0;           // uniaxial anisotropy constant (J/m^3)
    double ku_axis[3] = {0.0, 0.0, 1.0};
    double stt_j = 0.0;        // Slonczewski torque: current density (A/m^2), 0 = none
    double stt_P = 0.0, stt_lambda = 1.0, stt_epsp = 0.0, stt_d = 1.0;
    double stt_p[3] = {0.0, 0.0, 1.0};
    hipStream_t stream = nullptr;
    int device = 0;
    // device memory
    std::vector<void *> allocs;
    size_t bytes = 0;
    void *S1 = nullptr, *S2 = nullptr, *tensor = nullptr, *twT = nullptr, *tw64 = nullptr;
    void *ms[2] = {nullptr, nullptr}, *acc = nullptr;
    double *epart = nullptr, *esum = nullptr;
    int st_cx = 0, st_nqb = 0, st_blocks = 0;   // stencil kernel of h_eff without demag (0: not applicable)
    LinePass *d_lp = nullptr;   // [0] y forward, [1] y inverse
    FusedPass *d_fp = nullptr;
    // host copies
    HostFft fx, fy, fz;
    std::vector<int> order[3];  // radix order per axis for the runtime-planned kernels (empty: default)
    size_t tw_off[3] = {0, 0, 0};   // offsets (complex units) of the x, y, z tables in twT
    LinePass lp_fwd{}, lp_inv{};
    FusedPass fp{};
    ZGeom zg{};
    size_t lds_fwd = 0, lds_inv = 0, lds_fp = 0, lds_z = 0;
    bool x_ct = false, y_ct = false, z_ct = false;   // power-of-two specialised kernels in use
    bool i32 = false;          // the compile-time z-inverse kernels may index cells and S1 in 32 bits
    int y_var = 0;                                   // specialised y pass: 0 LDS-resident pencil, 1 register-resident
    int x_var[2] = {0, 0};                          // variants of the forward / inverse x pass (0, 1: tile widths; 2: half-LDS; 3: half-LDS, wide tiles)
    int tiles_fwd = 0, tiles_inv = 0;
    // llg graph cache; graphs are captured on a private stream (capture is not
    // permitted on the legacy default stream) and launched on `stream`
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<unsigned char> gkey;
    // scratch of the RK4 step's adjoint (14 vector fields), of the RKF45
    // step (6 stage derivatives and the candidate) and of the minimiser
    // (previous m, two gradient fields, per-block and total sums): one region
    // that each of them uses only within one call, in stream order.  Either
    // caller-owned (mm_plan_attach_scratch) or, for a plan that owns its
    // memory, allocated on first use and grown when a call needs more.
    void *scr = nullptr;
    size_t scr_bytes = 0;
    bool scr_ext = false;
    // orders a newly set stream after the work enqueued on the previous one
    hipEvent_t ev = nullptr;
    // memory sizing and caller-owned memory: a dry plan only adds up sizes;
    // with a workspace attached, allocations are carved from it and the tensor
    // spectrum lives in the caller's tensor buffer
    bool dry = false;
    size_t ws_used = 0, tensor_bytes = 0;
    char *ws = nullptr;
    void *tensor_ext = nullptr;
};

namespace {

int dalloc_own(mm_plan *p, void **out, size_t bytes);

// plan memory: carved from the attached workspace, counted in a dry plan,
// else allocated by the plan
int dalloc(mm_plan *p, void **out, size_t bytes) {
    *out = nullptr;
    if (bytes == 0) bytes = 256;
    if (p->dry || p->ws) {
        // sub-buffers of the workspace start on 256-byte boundaries
        const size_t off = (p->ws_used + 255) & ~(size_t)255;
        p->ws_used = off + bytes;
        if (p->ws) *out = p->ws + off;
        return MM_OK;
    }
    return dalloc_own(p, out, bytes);
}

// memory the plan allocates and frees itself
int dalloc_own(mm_plan *p, void **out, size_t bytes) {
    *out = nullptr;
    if (bytes == 0) bytes = 256;
    if (getenv("MMX_TEST_FAIL_ALLOC")) return fail(MM_ENOMEM, "allocation of %zu bytes refused (MMX_TEST_FAIL_ALLOC)", bytes);
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) {
        *out = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? MM_ENOMEM : MM_EHIP, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    p->allocs.push_back(*out);
    p->bytes += bytes;
    return MM_OK;
}

void free_all(mm_plan *p) {
    if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
    if (p->cap) { (void)hipStreamDestroy(p->cap); p->cap = nullptr; }
    for (void *q : p->allocs) (void)hipFree(q);
    p->allocs.clear();
    if (!p->scr_ext) { p->scr = nullptr; p->scr_bytes = 0; }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// blocks of the z-inverse pass (its per-block reduction partials)
int zinv_tiles(const mm_plan *p) {
    return p->z_ct ? zinv_ct_tiles(p->zg.nx, p->zg.ny, p->zg.Lz, p->zg.ygrp) : p->zg.tiles;
}

// Scratch bytes of the entry points that need more than the plan's workspace:
// [0] llg_step_adjoint, [1] llg_rkf45_step, [2] mm_minimize_bb.
void scratch_need(int64_t ncell, size_t rsz, int tiles, size_t out[3]) {
    const size_t f3 = (size_t)ncell * 3 * rsz;
    out[0] = 14 * f3;
    out[1] = 7 * f3;
    out[2] = 3 * align256(f3) + align256((size_t)tiles * 4 * sizeof(double)) + 4 * sizeof(double);
}

// the scratch region for a call that needs `need` bytes
int get_scratch(mm_plan *p, size_t need, void **out) {
    *out = nullptr;
    if (p->scr && p->scr_bytes >= need) { *out = p->scr; return MM_OK; }
    if (p->scr_ext || p->ws)
        return fail(MM_ESTATE, "this call needs %zu bytes of scratch memory and the plan has %zu attached "
                               "(mm_plan_scratch_bytes, mm_plan_attach_scratch)", need, p->scr_ext ? p->scr_bytes : (size_t)0);
    if (p->scr) {
        // grow: work still queued may use the old region
        HIPCK(hipStreamSynchronize(p->stream));
        auto it = std::find(p->allocs.begin(), p->allocs.end(), p->scr);
        if (it != p->allocs.end()) p->allocs.erase(it);
        (void)hipFree(p->scr);
        p->bytes -= p->scr_bytes;
        p->scr = nullptr;
        p->scr_bytes = 0;
    }
    int rc = dalloc_own(p, &p->scr, need);
    if (rc) return rc;
    p->scr_bytes = need;
    *out = p->scr;
    return MM_OK;
}

template <typename T>
std::vector<T> round_tw(const HostFft &f) {
    std::vector<T> v(f.tw.size());
    for (size_t i = 0; i < v.size(); ++i) v[i] = (T)f.tw[i];
    return v;
}

// Tile choice for a line pass of length L: columns W (power of two) within the
// LDS budget, at most `inner`, with the FFT fitting 1024 threads.
// Tile choice for a line pass of length L: the first candidate width (all
// `inner` columns if few, else 64, 32, ..., 1) that fits the LDS budget and
// 1024 threads; `want_W` > 0 forces a width (clamped to `inner`).
void choose_line_tile(int L, int inner, size_t csz, size_t budget, int want_W, int &W, int &nthr, size_t &lds) {
    const int pitch = pitch_of(L);
    const FftDesc d = make_fft(L).d;
    std::vector<int> cand;
    if (want_W > 0) cand.push_back(std::min(want_W, inner));
    if (inner <= 64) cand.push_back(inner);
    for (int w = 64; w >= 1; w >>= 1)
        if (w <= inner) cand.push_back(w);
    W = 1;
    for (int w : cand) {
        if ((size_t)w * pitch * csz <= budget && fft_threads(d, w, w * L) <= 1024) { W = w; break; }
    }
    nthr = fft_threads(d, W, W * L);
    lds = (size_t)W * pitch * csz;
}

int validate_grid(const int64_t grid[3], const double cell[3]) {
    if (!grid || !cell) return fail(MM_EINVAL, "grid and cell must be non-NULL");
    for (int a = 0; a < 3; ++a) {
        if (grid[a] < 1 || grid[a] > (1 << 20)) return fail(MM_EINVAL, "grid[%d]=%lld out of range [1, 2^20]", a, (long long)grid[a]);
        if (!(cell[a] > 0.0) || !std::isfinite(cell[a])) return fail(MM_EINVAL, "cell[%d] must be finite and > 0", a);
    }
    return MM_OK;
}

template <typename T> int build_spectrum(mm_plan *p, const double *d_octant);

// set up the FFT descriptors, tiles and workspace of a plan
template <typename T>
int setup_plan(mm_plan *p, const mm_plan_opts *o) {
    typedef cplx<T> C;
    const size_t csz = sizeof(C);
    const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
    const int Lx = (int)p->L[0], Ly = (int)p->L[1], Lz = (int)p->L[2];
    p->hx = Lx / 2 + 1;
    p->hy = Ly / 2 + 1;
    p->hz = Lz / 2 + 1;
    // test hook: MMX_ORDER="x:4,5,5;y:2,3,3,5" sets the radix order of
    // runtime-planned (non-power-of-two) axes; a list that is not a
    // permutation of the length's factors is ignored
    if (const char *e = getenv("MMX_ORDER")) {
        std::string t(e);
        for (size_t i = 0; i + 2 <= t.size();) {
            const size_t end = std::min(t.find(';', i), t.size());
            const int a = t[i] == 'x' ? 0 : t[i] == 'y' ? 1 : t[i] == 'z' ? 2 : -1;
            if (a >= 0 && t[i + 1] == ':' && (p->L[a] & (p->L[a] - 1)) != 0) {
                std::vector<int> o = parse_order(t.substr(i + 2, end - i - 2));
                std::vector<int> f = factorize((int)p->L[a]), q = o;
                std::sort(f.begin(), f.end());
                std::sort(q.begin(), q.end());
                if (q == f) p->order[a] = o;
            }
            i = end + 1;
        }
    }
    p->fx = make_fft(Lx, false, p->order[0]);
    p->fy = make_fft(Ly, false, p->order[1]);
    p->fz = make_fft(Lz, false, p->order[2]);
    // twiddles (plan precision): x, y, z tables concatenated
    std::vector<T> tw;
    auto app = [&](const HostFft &f) { size_t off = tw.size() / 2; auto v = round_tw<T>(f); tw.insert(tw.end(), v.begin(), v.end()); return off; };
    const size_t ox = app(p->fx), oy = app(p->fy);
    (void)app(make_fft(Ly, true));   // reversed radix order, right after y's table (fused inverse)
    // the Ly roots exp(-2 pi i m / Ly): twiddles of either radix order by index
    const size_t oroots = tw.size() / 2;
    for (int m = 0; m < Ly; ++m) {
        const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)Ly;
        tw.push_back((T)cosl(ang));
        tw.push_back((T)sinl(ang));
    }
    // stage-ordered tables of Ly/2 (forward, then reversed order) for the
    // fused pass in two half-spectra
    size_t ohalf = 0;
    if (fused_pf_available(Ly, 6)) {
        ohalf = app(make_fft(Ly / 2, false));
        (void)app(make_fft(Ly / 2, true));
    }
    const size_t oz = app(p->fz);
    p->tw_off[0] = ox; p->tw_off[1] = oy; p->tw_off[2] = oz;
    // folded z transform (compile-time Lz): table of length Lz/2, then exp(-2 pi i k / Lz), k <= Lz/2
    size_t ozh = 0;
    if (zct_cols(Lz) > 0) {
        ozh = app(make_fft(Lz / 2));
        for (int k = 0; k <= Lz / 2; ++k) {
            const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)Lz;
            tw.push_back((T)cosl(ang));
            tw.push_back((T)sinl(ang));
        }
    }
    int rc;
    if ((rc = dalloc(p, &p->twT, std::max<size_t>(tw.size() * sizeof(T), 16)))) return rc;
    if (!p->dry) HIPCK(hipMemcpy(p->twT, tw.data(), tw.size() * sizeof(T), hipMemcpyHostToDevice));
    const C *twc = reinterpret_cast<const C *>(p->twT);
    // workspace: S1 [kz][x][y][c] (kz < hz), S2 [kz][kx][y][c] (kx < Lx), tensor
    const int64_t npos = nx * ny;
    const size_t s1 = (size_t)p->hz * npos * 3 * csz, s2 = (size_t)p->hz * Lx * ny * 3 * csz;
    const size_t tens = (size_t)p->hz * p->hx * p->hy * 6 * sizeof(T);
    const size_t cells3 = (size_t)nx * ny * nz * 3 * sizeof(T);
    if ((rc = dalloc(p, &p->S1, s1))) return rc;
    if ((rc = dalloc(p, &p->S2, s2))) return rc;
    p->tensor_bytes = tens;
    if (p->dry) p->tensor = nullptr;
    else if (p->tensor_ext) p->tensor = p->tensor_ext;
    else if ((rc = dalloc(p, &p->tensor, tens))) return rc;
    if ((rc = dalloc(p, &p->ms[0], cells3))) return rc;
    if ((rc = dalloc(p, &p->ms[1], cells3))) return rc;
    if ((rc = dalloc(p, &p->acc, cells3))) return rc;
    // x passes: lines along x, columns (y, c) contiguous, one kz plane per outer index
    const int64_t ny3 = ny * 3;
    int W, nthr;
    size_t lds;
    choose_line_tile(Lx, (int)ny3, csz, kLdsTarget, 0, W, nthr, lds);
    int Wct = 0, NTct = 0;
    if (getenv("MMX_XVAR")) p->x_var[0] = p->x_var[1] = std::min(3, std::max(0, atoi(getenv("MMX_XVAR"))));
    if (p->x_var[0] == 3 && !line_ct_shape(Lx, csz, 3, &Wct, &NTct)) p->x_var[0] = p->x_var[1] = 2;   // no wide tiles
    // the specialised kernels address one kz plane (Lx rows) through a buffer
    // resource, whose size is a 31-bit byte count
    p->x_ct = line_ct_shape(Lx, csz, p->x_var[0], &Wct, &NTct) &&
              (p->x_var[0] >= 2 ? line_hx_lds(Lx, Wct, csz) : line_ct_lds(Lx, Wct, csz)) <= kLdsMax &&
              (int64_t)Lx * ny3 * (int64_t)csz < (int64_t(1) << 31) && !getenv("MMX_NO_CT");
    if (p->x_ct) { W = Wct; nthr = NTct; lds = p->x_var[0] >= 2 ? line_hx_lds(Lx, W, csz) : line_ct_lds(Lx, W, csz); }
    LinePass &f = p->lp_fwd;
    std::memset(&f, 0, sizeof f);
    f.in = p->S1; f.out = p->S2; f.tw = twc + ox;
    f.in_row = ny3; f.out_row = ny3; f.in_outer = nx * ny3; f.out_outer = (int64_t)Lx * ny3;
    f.inner = (int)ny3; f.outer = p->hz; f.n_in = (int)nx; f.n_out = Lx;
    f.W = W; f.tiles_inner = (int)((ny3 + W - 1) / W); f.pitch = p->x_ct ? Lx + 1 : pitch_of(Lx); f.nthr = nthr; f.sym_axis = -1;
    f.f = p->fx.d;
    p->lds_fwd = lds;
    p->tiles_fwd = f.tiles_inner * f.outer;
    LinePass &g = p->lp_inv;
    g = f;
    g.in = p->S2; g.out = p->S1; g.in_outer = (int64_t)Lx * ny3; g.out_outer = nx * ny3; g.n_in = Lx; g.n_out = (int)nx;
    p->lds_inv = lds;
    p->tiles_inv = p->tiles_fwd;
    // fused y pass: one (kz, kx) pencil of three components per tile
    FusedPass &q = p->fp;
    std::memset(&q, 0, sizeof q);
    const int npen = p->hz * Lx;
    const int py = pitch_of(Ly);
    int Wp = 1;
    for (int w : {8, 4, 2, 1}) {
        if (w <= std::max(1, npen) && (size_t)3 * w * py * csz <= kLdsTarget && fft_threads(p->fy.d, 3 * w, 3 * w * Ly) <= 1024) { Wp = w; break; }
    }
    // a y length whose LDS pencil does not fit one workgroup runs as two
    // half-spectra (variant 6, half the LDS) where that kernel has it
    const bool y_full = fused_ct_lds(Ly, csz) <= kLdsMax;
    const bool y_half = fused_pf_available(Ly, 6) && fused_ct_lds(Ly / 2, csz) <= kLdsMax;
    p->y_ct = fused_ct_threads(Ly, csz) > 0 && (y_full || y_half) && !getenv("MMX_NO_CT");
    if (p->y_ct && !y_full) p->y_var = 6;
    if (p->y_ct && y_full && getenv("MMX_YVAR")) {
        const int v = atoi(getenv("MMX_YVAR"));
        if ((v == 1 && fused_hx_threads(Ly) > 0) || fused_pf_available(Ly, v)) p->y_var = v;
    }
    if (p->y_ct) Wp = 1;
    q.data = p->S2; q.tensor = p->tensor; q.tw = twc + oy; q.roots = twc + oroots; q.twh = ohalf ? twc + ohalf : nullptr;
    q.n = (int)ny; q.Lx = Lx; q.Ly = Ly; q.hz = p->hz; q.hxp = p->hx; q.hyp = p->hy;
    q.npos = npen; q.W = Wp; q.tiles = (npen + Wp - 1) / Wp;
    q.pitch = p->y_ct ? Ly + 1 : py;
    q.nthr = p->y_ct ? fused_ct_threads(Ly, csz) : fft_threads(p->fy.d, 3 * Wp, 3 * Wp * Ly);
    q.f = p->fy.d;
    p->lds_fp = p->y_ct ? fused_ct_lds(y_full ? Ly : Ly / 2, csz) : (size_t)3 * Wp * q.pitch * csz;
    if (p->lds_fp > kLdsMax) return fail(MM_ENOTSUP, "y length %d too long for one workgroup", Ly);
    // z passes: P positions (even) per tile, about 512 cells per tile
    ZGeom &z = p->zg;
    std::memset(&z, 0, sizeof z);
    z.nx = (int)nx; z.ny = (int)ny; z.nz = (int)nz; z.Lz = Lz; z.hz = p->hz;
    const int pz = pitch_of(Lz);
    int P = (int)std::max<int64_t>(2, (1024 / nz) & ~1);
    P = std::min<int64_t>(P, std::max<int64_t>(2, (nx * ny + 1) & ~1));
    while (P > 2 && ((size_t)((3 * P + 1) / 2) * pz * csz > 48 * 1024 || fft_threads(p->fz.d, (3 * P + 1) / 2, P * (int)nz) > 1024)) P -= 2;
    p->z_ct = zct_cols(Lz) > 0 && !getenv("MMX_NO_CT");
    if (p->z_ct) P = zct_cols(Lz);
    z.P = P; z.tiles = (int)((nx * ny + P - 1) / P); z.pitch = pz;
    z.dnz = make_fastdiv((uint32_t)nz); z.dny = make_fastdiv((uint32_t)ny);
    z.nthr = std::min(1024, std::max(256, fft_threads(p->fz.d, (3 * P + 1) / 2, P * (int)nz)));
    z.f = p->fz.d; z.tw = twc + oz; z.twh = twc + ozh; z.S1 = p->S1;
    p->lds_z = std::max<size_t>((size_t)((3 * P + 1) / 2) * pz * csz, 16 * 4 * sizeof(double) + 64);
    if (p->z_ct) p->lds_z = std::max(p->lds_z, zct_lds(Lz, csz));
    // grouped z-inverse tile order for the compile-time kernels (x
    // neighbours' rows read while still in L2); linear runs for short rows
    z.ygrp = (p->z_ct && ny >= P) ? (int)std::min<int64_t>(4, (ny + P - 1) / P) : 0;
    if ((size_t)((3 * P + 1) / 2) * pz * csz > kLdsMax) return fail(MM_ENOTSUP, "z length %d too long", Lz);
    // energy partials
    if ((rc = dalloc(p, (void **)&p->epart, (size_t)std::max(z.tiles, zinv_tiles(p)) * 2 * sizeof(double)))) return rc;
    if (!stencil_shape((int)p->n[0], (int)p->n[1], (int)p->n[2], z.tiles, &p->st_cx, &p->st_nqb, &p->st_blocks))
        p->st_blocks = 0;
    if ((rc = dalloc(p, (void **)&p->esum, 2 * sizeof(double)))) return rc;
    // device descriptor copies
    if ((rc = dalloc(p, (void **)&p->d_lp, 2 * sizeof(LinePass)))) return rc;
    if ((rc = dalloc(p, (void **)&p->d_fp, sizeof(FusedPass)))) return rc;
    LinePass two[2] = {p->lp_fwd, p->lp_inv};
    if (!p->dry) {
        HIPCK(hipMemcpy(p->d_lp, two, sizeof two, hipMemcpyHostToDevice));
        HIPCK(hipMemcpy(p->d_fp, &p->fp, sizeof(FusedPass), hipMemcpyHostToDevice));
    }
    // FP64 twiddles for the tensor transforms
    std::vector<double> tw64;
    auto app64 = [&](const HostFft &h) { size_t off = tw64.size() / 2; auto v = round_tw<double>(h); tw64.insert(tw64.end(), v.begin(), v.end()); return off; };
    (void)app64(p->fx); (void)app64(p->fy); (void)app64(p->fz);
    if ((rc = dalloc(p, &p->tw64, std::max<size_t>(tw64.size() * sizeof(double), 16)))) return rc;
    if (!p->dry) HIPCK(hipMemcpy(p->tw64, tw64.data(), tw64.size() * sizeof(double), hipMemcpyHostToDevice));
    return MM_OK;
}

// One real symmetric (cosine / sine) transform pass of the FP64 tensor.
int sym_pass(mm_plan *p, const double *in, double *out, int axis, int64_t outer, int inner, int64_t in_row,
             int64_t in_outer, int64_t out_row, int64_t out_outer, int n_in, int L, const HostFft &hf,
             const double2 *tw, void *d_desc) {
    int W, nthr;
    size_t lds;
    choose_line_tile(L, inner, sizeof(double2), kLdsTarget, 0, W, nthr, lds);
    LinePass a;
    std::memset(&a, 0, sizeof a);
    a.in = in; a.out = out; a.tw = tw;
    a.in_row = in_row; a.out_row = out_row; a.in_outer = in_outer; a.out_outer = out_outer;
    a.inner = inner; a.outer = (int)outer; a.n_in = n_in; a.n_out = L / 2 + 1;
    a.W = W; a.tiles_inner = (inner + W - 1) / W; a.pitch = pitch_of(L); a.nthr = nthr; a.sym_axis = axis;
    a.f = hf.d;
    HIPCK(hipMemcpyAsync(d_desc, &a, sizeof a, hipMemcpyHostToDevice, p->stream));
    const long long tiles = (long long)a.tiles_inner * outer;
    if (tiles > 0x7fffffffLL) return fail(MM_ENOTSUP, "tensor transform grid too large");
    HIPCK(launch_line_pass<double>((const LinePass *)d_desc, nullptr, (int)tiles, nthr, lds, -1, true, p->stream));
    HIPCK(hipStreamSynchronize(p->stream));
    return MM_OK;
}

// real-space FP64 octant (device) -> stored spectrum in plan precision
template <typename T>
int build_spectrum(mm_plan *p, const double *d_oct) {
    const int64_t nx = p->n[0], ny = p->n[1], nz = p->n[2];
    const int Lx = (int)p->L[0], Ly = (int)p->L[1], Lz = (int)p->L[2];
    const int hx = p->hx, hy = p->hy, hz = p->hz;
    const size_t big = (size_t)std::max<int64_t>(nx, hx) * std::max<int64_t>(ny, hy) * std::max<int64_t>(nz, hz) * 6 * sizeof(double);
    void *b0 = nullptr, *b1 = nullptr, *dd = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&b0, big)) != hipSuccess) return fail(MM_ENOMEM, "tensor scratch: %s", hipGetErrorString(e));
    if ((e = hipMalloc(&b1, big)) != hipSuccess) { (void)hipFree(b0); return fail(MM_ENOMEM, "tensor scratch: %s", hipGetErrorString(e)); }
    if ((e = hipMalloc(&dd, sizeof(LinePass))) != hipSuccess) { (void)hipFree(b0); (void)hipFree(b1); return fail(MM_ENOMEM, "desc"); }
    const double2 *tw = reinterpret_cast<const double2 *>(p->tw64);
    const size_t ox = 0, oy = (size_t)std::max(p->fx.d.L - 1, 0), oz = oy + (size_t)std::max(p->fy.d.L - 1, 0);
    int rc = MM_OK;
    // z: [i][j][k][q] -> [i][j][kz][q]
    rc = sym_pass(p, d_oct, (double *)b0, 2, nx * ny, 6, 6, nz * 6, 6, (int64_t)hz * 6, (int)nz, Lz, p->fz, tw + oz, dd);
    // y: [i][j][kz][q] -> [i][ky][kz][q]
    if (!rc) rc = sym_pass(p, (double *)b0, (double *)b1, 1, nx, hz * 6, (int64_t)hz * 6, ny * hz * 6, (int64_t)hz * 6,
                           (int64_t)hy * hz * 6, (int)ny, Ly, p->fy, tw + oy, dd);
    // x: [i][ky][kz][q] -> [kx][ky][kz][q]
    if (!rc) rc = sym_pass(p, (double *)b1, (double *)b0, 0, 1, hy * hz * 6, (int64_t)hy * hz * 6, 0, (int64_t)hy * hz * 6,
                           0, (int)nx, Lx, p->fx, tw + ox, dd);
    if (!rc) {
        const double inv = 1.0 / ((double)Lx * Ly * Lz);
        hipError_t le = launch_tensor_finalize<T>((const double *)b0, (T *)p->tensor, hx, hy, hz, inv, p->stream);
        if (le != hipSuccess) rc = fail(MM_EHIP, "tensor finalize: %s", hipGetErrorString(le));
        else if ((le = hipStreamSynchronize(p->stream)) != hipSuccess) rc = fail(MM_EHIP, "tensor: %s", hipGetErrorString(le));
    }
    (void)hipFree(b0); (void)hipFree(b1); (void)hipFree(dd);
    return rc;
}

// one specialised x pass (dir -1 forward, +1 inverse) in the plan's variant
template <typename T>
hipError_t launch_x(mm_plan *p, int dir) {
    const LinePass &a = dir < 0 ? p->lp_fwd : p->lp_inv;
    const int v = p->x_var[dir < 0 ? 0 : 1];
    const int tiles = dir < 0 ? p->tiles_fwd : p->tiles_inv;
    if (v == 3) return launch_line_wide<T>(a, tiles, a.W, dir, p->stream);
    return launch_line_ct<T>(a, tiles, a.W, dir, p->stream, v == 2 ? 1 : 0);
}

// the specialised fused y pass in the plan's variant
template <typename T>
hipError_t launch_y(mm_plan *p) {
    if (p->y_var >= 2) return launch_fused_pf<T>(p->fp, p->y_var, p->stream);
    return p->y_var == 1 ? launch_fused_hx<T>(p->fp, p->stream) : launch_fused_ct<T>(p->fp, p->stream);
}

// the fused y pass variants a plan of y length Ly can run
std::vector<int> y_variants(int Ly, size_t csz) {
    if (fused_ct_lds(Ly, csz) > kLdsMax) return fused_pf_available(Ly, 6) ? std::vector<int>{6} : std::vector<int>{};
    std::vector<int> v{0};
    if (fused_hx_threads(Ly) > 0) v.push_back(1);
    for (int k = 2; k <= 6; ++k)
        if (fused_pf_available(Ly, k)) v.push_back(k);
    return v;
}

// Switch the forward (d = 0) or inverse (d = 1) specialised x pass to
// variant v (descriptor, LDS).
int configure_x(mm_plan *p, int d, int v) {
    const size_t csz = p->prec == MM_F32 ? sizeof(float2) : sizeof(double2);
    int W = 0, NT = 0;
    if (!p->x_ct || !line_ct_shape((int)p->L[0], csz, v, &W, &NT)) return MM_OK;
    p->x_var[d] = v;
    LinePass *f = d == 0 ? &p->lp_fwd : &p->lp_inv;
    f->W = W;
    f->nthr = NT;
    f->tiles_inner = (f->inner + W - 1) / W;
    const size_t lds = v >= 2 ? line_hx_lds((int)p->L[0], W, csz) : line_ct_lds((int)p->L[0], W, csz);
    (d == 0 ? p->lds_fwd : p->lds_inv) = lds;
    (d == 0 ? p->tiles_fwd : p->tiles_inv) = f->tiles_inner * f->outer;
    LinePass two[2] = {p->lp_fwd, p->lp_inv};
    HIPCK(hipMemcpy(p->d_lp, two, sizeof two, hipMemcpyHostToDevice));
    return MM_OK;
}

int configure_x(mm_plan *p, int v) {
    int rc = configure_x(p, 0, v);
    return rc ? rc : configure_x(p, 1, v);
}

// ---- autotuner -------------------------------------------------------------
// Launch schedules (x and y pass kernel variants, radix orders of the
// runtime-planned transforms) are timed on the plan's own buffers and the
// winners recorded in a schedule cache keyed by device, precision, pass,
// transform length and problem size (log2 of the points a launch
// transforms).  Modes: 0 off (default schedules), 1 cached (take a recorded
// winner, time the candidates on a miss), 2 search (always time; record).
// MMX_AUTOTUNE=off|cached|search overrides the plan option;
// MMX_AUTOTUNE_CACHE=<file> keeps the cache across processes (one
// "key<TAB>value" line per entry, appended as winners are found).
enum { TUNE_OFF = 0, TUNE_CACHED = 1, TUNE_SEARCH = 2 };

struct TuneCache {
    std::mutex mu;
    std::map<std::string, std::string> kv;
    bool loaded = false;
    std::string path;
};

TuneCache &tune_cache() {
    static TuneCache c;
    return c;
}

// (re)read the cache file when MMX_AUTOTUNE_CACHE names a file not read yet
void tune_load_locked(TuneCache &c) {
    const char *f = getenv("MMX_AUTOTUNE_CACHE");
    const std::string path = f ? f : "";
    if (c.loaded && path == c.path) return;
    c.loaded = true;
    c.path = path;
    if (path.empty()) return;
    FILE *fp = fopen(path.c_str(), "r");
    if (!fp) return;
    char line[512];
    while (fgets(line, sizeof line, fp)) {
        char *tab = strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        std::string v(tab + 1);
        while (!v.empty() && (v.back() == '\n' || v.back() == '\r')) v.pop_back();
        c.kv[line] = v;
    }
    fclose(fp);
}

bool tune_get(const std::string &k, std::string &v) {
    TuneCache &c = tune_cache();
    std::lock_guard<std::mutex> g(c.mu);
    tune_load_locked(c);
    auto it = c.kv.find(k);
    if (it == c.kv.end()) return false;
    v = it->second;
    return true;
}

void tune_put(const std::string &k, const std::string &v) {
    TuneCache &c = tune_cache();
    std::lock_guard<std::mutex> g(c.mu);
    tune_load_locked(c);
    c.kv[k] = v;
    if (!c.path.empty()) {
        FILE *fp = fopen(c.path.c_str(), "a");
        if (fp) { fprintf(fp, "%s\t%s\n", k.c_str(), v.c_str()); fclose(fp); }
    }
}

int tune_mode(int opt) {
    const char *e = getenv("MMX_AUTOTUNE");
    if (e && !strcmp(e, "off")) return TUNE_OFF;
    if (e && !strcmp(e, "cached")) return TUNE_CACHED;
    if (e && !strcmp(e, "search")) return TUNE_SEARCH;
    return opt;
}

// "<arch>/<CUs>" of a device, looked up once per device
std::string device_tag(int dev) {
    static std::mutex mu;
    static std::map<int, std::string> tags;
    std::lock_guard<std::mutex> g(mu);
    auto it = tags.find(dev);
    if (it != tags.end()) return it->second;
    hipDeviceProp_t prop;
    std::string t = "dev";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        std::string arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch.resize(colon);
        t = arch + "/" + std::to_string(prop.multiProcessorCount);
    }
    tags[dev] = t;
    return t;
}

std::string tune_key(int dev, int prec, const char *what, int L, long long points) {
    int b = 0;
    while (b < 62 && (1LL << (b + 1)) <= points) ++b;
    char buf[160];
    snprintf(buf, sizeof buf, "%s %s %s L%d p2^%d", device_tag(dev).c_str(), prec == MM_F32 ? "f32" : "f64", what, L, b);
    return buf;
}

// ms of three back-to-back launches, best of two repetitions
template <class F>
int time3(hipStream_t s, hipEvent_t e0, hipEvent_t e1, F launch, float *best) {
    *best = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
        HIPCK(hipEventRecord(e0, s));
        for (int k = 0; k < 3; ++k) {
            hipError_t e = launch();
            if (e != hipSuccess) return fail(MM_EHIP, "autotune: %s", hipGetErrorString(e));
        }
        HIPCK(hipEventRecord(e1, s));
        HIPCK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCK(hipEventElapsedTime(&ms, e0, e1));
        *best = std::min(*best, ms);
    }
    return MM_OK;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    int make() {
        HIPCK(hipEventCreate(&a));
        HIPCK(hipEventCreate(&b));
        return MM_OK;
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// the x pass variants a plan can run (LDS permitting)
std::vector<int> x_variants(const mm_plan *p) {
    std::vector<int> v;
    if (!p->x_ct) return v;
    const size_t csz = p->prec == MM_F32 ? sizeof(float2) : sizeof(double2);
    for (int k = 0; k < 4; ++k) {
        int W = 0, NT = 0;
        if (!line_ct_shape((int)p->L[0], csz, k, &W, &NT)) continue;
        if ((k >= 2 ? line_hx_lds((int)p->L[0], W, csz) : line_ct_lds((int)p->L[0], W, csz)) > kLdsMax) continue;
        v.push_back(k);
    }
    return v;
}

// Forward and inverse x pass variants.
template <typename T>
int autotune_x(mm_plan *p, int mode) {
    const std::vector<int> cand = x_variants(p);
    if (cand.size() < 2) return MM_OK;
    EventPair ev;
    int rc = ev.make();
    const long long pts = (long long)p->hz * p->n[1] * 3 * p->L[0];
    for (int d = 0; d < 2 && !rc; ++d) {
        const std::string key = tune_key(p->device, p->prec, d == 0 ? "x_fwd" : "x_inv", (int)p->L[0], pts);
        std::string got;
        if (mode == TUNE_CACHED && tune_get(key, got)) {
            const int v = atoi(got.c_str());
            if (std::find(cand.begin(), cand.end(), v) != cand.end()) { rc = configure_x(p, d, v); continue; }
        }
        float best = 1e30f;
        int bestv = p->x_var[d];
        for (int v : cand) {
            if ((rc = configure_x(p, d, v))) break;
            float ms = 0.f;
            if ((rc = time3(p->stream, ev.a, ev.b, [&] { return launch_x<T>(p, d == 0 ? -1 : +1); }, &ms))) break;
            if (ms < best) { best = ms; bestv = v; }
        }
        if (!rc) rc = configure_x(p, d, bestv);
        if (!rc) tune_put(key, std::to_string(bestv));
    }
    return rc;
}

// Fused y pass variants: the LDS-resident, register-resident, wave-rotated
// and persistent (next pencil's loads in flight) pencil kernels.
template <typename T>
int autotune_y(mm_plan *p, int mode) {
    const std::vector<int> cand = y_variants((int)p->L[1], 2 * p->rsz);
    if (!p->y_ct || cand.size() < 2) return MM_OK;
    const std::string key = tune_key(p->device, p->prec, "y_fused", (int)p->L[1], (long long)p->fp.npos * p->L[1]);
    std::string got;
    if (mode == TUNE_CACHED && tune_get(key, got)) {
        const int v = atoi(got.c_str());
        if (std::find(cand.begin(), cand.end(), v) != cand.end()) { p->y_var = v; return MM_OK; }
    }
    EventPair ev;
    int rc = ev.make();
    float best = 1e30f;
    int bestv = p->y_var;
    for (int v : cand) {
        if (rc) break;
        p->y_var = v;
        float ms = 0.f;
        if ((rc = time3(p->stream, ev.a, ev.b, [&] { return launch_y<T>(p); }, &ms))) break;
        if (ms < best) { best = ms; bestv = v; }
    }
    p->y_var = bestv;
    if (!rc) tune_put(key, std::to_string(bestv));
    return rc;
}

// Candidate radix orders of a runtime-planned transform: every distinct
// permutation of the factors when there are at most 24, else the default
// order, its reverse, its rotations and the two sorted orders.
std::vector<std::vector<int>> radix_orders(int L) {
    std::vector<int> f = factorize(L);
    std::vector<std::vector<int>> out;
    std::vector<int> s = f;
    std::sort(s.begin(), s.end());
    long long count = 0;
    do { ++count; } while (count <= 24 && std::next_permutation(s.begin(), s.end()));
    std::sort(s.begin(), s.end());
    auto add = [&](const std::vector<int> &o) {
        if (std::find(out.begin(), out.end(), o) == out.end()) out.push_back(o);
    };
    add(f);
    if (count <= 24) {
        do { add(s); } while (std::next_permutation(s.begin(), s.end()));
    } else {
        std::vector<int> r = f;
        std::reverse(r.begin(), r.end());
        add(r);
        for (size_t k = 1; k < f.size(); ++k) {
            std::vector<int> q(f.begin() + k, f.end());
            q.insert(q.end(), f.begin(), f.begin() + k);
            add(q);
        }
        add(s);
        std::reverse(s.begin(), s.end());
        add(s);
    }
    return out;
}

std::string order_str(const std::vector<int> &o) {
    std::string r;
    for (size_t i = 0; i < o.size(); ++i) r += (i ? "," : "") + std::to_string(o[i]);
    return r;
}

// Install radix order `o` for axis a of a runtime-planned pass: the host
// descriptor, the twiddle table in place (its size, L-1, does not depend on
// the order) and the device copies of the pass descriptors.
template <typename T>
int set_order(mm_plan *p, int a, const std::vector<int> &o) {
    const int L = (int)p->L[a];
    HostFft h = make_fft(L, false, o);
    std::vector<T> tw = round_tw<T>(h);
    if ((int)tw.size() != 2 * (L - 1)) return fail(MM_EINVAL, "radix order does not factor L=%d", L);
    cplx<T> *base = reinterpret_cast<cplx<T> *>(p->twT) + p->tw_off[a];
    HIPCK(hipMemcpy(base, tw.data(), tw.size() * sizeof(T), hipMemcpyHostToDevice));
    // the FP64 table of the tensor transforms (x, y, z tables of L-1 entries
    // each) follows the new order too, so that a later mm_demag_tensor_set
    // builds the spectrum with matching descriptors and twiddles
    const std::vector<double> tw64 = round_tw<double>(h);
    size_t off64 = 0;
    for (int b = 0; b < a; ++b) off64 += (size_t)std::max<int64_t>(p->L[b] - 1, 0);
    HIPCK(hipMemcpy(reinterpret_cast<double2 *>(p->tw64) + off64, tw64.data(), tw64.size() * sizeof(double),
                    hipMemcpyHostToDevice));
    p->order[a] = o;
    if (a == 0) {
        p->fx = h;
        p->lp_fwd.f = h.d;
        p->lp_inv.f = h.d;
        LinePass two[2] = {p->lp_fwd, p->lp_inv};
        HIPCK(hipMemcpy(p->d_lp, two, sizeof two, hipMemcpyHostToDevice));
    } else if (a == 1) {
        p->fy = h;
        p->fp.f = h.d;
        HIPCK(hipMemcpy(p->d_fp, &p->fp, sizeof(FusedPass), hipMemcpyHostToDevice));
    } else {
        p->fz = h;
        p->zg.f = h.d;
    }
    return MM_OK;
}

template <typename T> int time_one(mm_plan *p, int k);

// Radix orders of the axes that run the runtime-planned kernels (lengths
// with two or more distinct radices), each timed on the passes along it.
template <typename T>
int autotune_radix(mm_plan *p, int mode) {
    const bool rt[3] = {!p->x_ct, !p->y_ct, !p->z_ct};
    EventPair ev;
    int rc = MM_OK;
    bool made = false;
    for (int a = 0; a < 3 && !rc; ++a) {
        if (!rt[a] || p->L[a] < 2) continue;
        const std::vector<std::vector<int>> cand = radix_orders((int)p->L[a]);
        if (cand.size() < 2) continue;
        static const char *what[3] = {"x_order", "y_order", "z_order"};
        const long long pts = (long long)p->n[0] * p->n[1] * p->n[2] * 8;
        const std::string key = tune_key(p->device, p->prec, what[a], (int)p->L[a], pts);
        std::string got;
        if (mode == TUNE_CACHED && tune_get(key, got)) {
            const std::vector<int> o = parse_order(got);
            if (std::find(cand.begin(), cand.end(), o) != cand.end()) { rc = set_order<T>(p, a, o); continue; }
        }
        if (!made) { if ((rc = ev.make())) break; made = true; }
        float best = 1e30f;
        std::vector<int> bo = cand[0];
        for (const std::vector<int> &o : cand) {
            if ((rc = set_order<T>(p, a, o))) break;
            float ms = 0.f;
            auto run = [&]() -> hipError_t {
                int r = MM_OK;
                if (a == 0) { r = time_one<T>(p, 1); if (!r) r = time_one<T>(p, 3); }
                else if (a == 1) r = time_one<T>(p, 2);
                else { r = time_one<T>(p, 0); if (!r) r = time_one<T>(p, 5); }
                return r ? hipErrorUnknown : hipSuccess;
            };
            if ((rc = time3(p->stream, ev.a, ev.b, run, &ms))) break;
            if (ms < best) { best = ms; bo = o; }
        }
        if (!rc) rc = set_order<T>(p, a, bo);
        if (!rc) tune_put(key, order_str(bo));
    }
    return rc;
}

int compute_tensor(mm_plan *p) {
    const size_t oct = (size_t)p->n[0] * p->n[1] * p->n[2] * 6 * sizeof(double);
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, oct);
    if (e != hipSuccess) return fail(MM_ENOMEM, "octant: %s", hipGetErrorString(e));
    e = launch_tensor_octant((double *)d, (int)p->n[0], (int)p->n[1], (int)p->n[2], p->d[0], p->d[1], p->d[2], p->P, p->stream);
    if (e != hipSuccess) { (void)hipFree(d); return fail(MM_EHIP, "tensor octant: %s", hipGetErrorString(e)); }
    int rc = p->prec == MM_F32 ? build_spectrum<float>(p, (double *)d) : build_spectrum<double>(p, (double *)d);
    (void)hipFree(d);
    return rc;
}

// ---- pass launchers --------------------------------------------------------
template <typename T>
int run_zfwd(mm_plan *p, int src, const void *srcp, const void *Ms, double Ms_s, const void *s = nullptr,
             const void *h = nullptr, const void *kb = nullptr, void *ym = nullptr, void *yh = nullptr, double gp = 0,
             double alpha = 0) {
    ZFwdArgs a;
    std::memset(&a, 0, sizeof a);
    a.g = p->zg; a.src = srcp; a.Ms = Ms; a.Ms_scalar = Ms_s;
    a.s = s; a.h = h; a.kb = kb; a.ym = ym; a.yh = yh; a.gp = gp; a.alpha = alpha;
    if (p->z_ct && src != SRC_ADJPRE) HIPCK(launch_zfwd_ct<T>(a, src, p->stream));
    else HIPCK(launch_zfwd<T>(a, src, p->lds_z, p->stream));
    return MM_OK;
}

template <typename T>
int run_xyx(mm_plan *p) {
    if (p->x_ct) HIPCK(launch_x<T>(p, -1));
    else HIPCK(launch_line_pass<T>(p->d_lp, nullptr, p->tiles_fwd, p->lp_fwd.nthr, p->lds_fwd, -1, false, p->stream));
    if (p->y_ct) HIPCK(launch_y<T>(p));
    else HIPCK(launch_fused_y<T>(p->d_fp, nullptr, p->fp.tiles, p->fp.nthr, p->lds_fp, p->stream));
    if (p->x_ct) HIPCK(launch_x<T>(p, +1));
    else HIPCK(launch_line_pass<T>(p->d_lp + 1, nullptr, p->tiles_inv, p->lp_inv.nthr, p->lds_inv, +1, false, p->stream));
    return MM_OK;
}

template <typename T>
hipError_t zinv_any(mm_plan *p, const ZInvArgs &a, int epi) {
    if (p->z_ct) return launch_zinv_ct<T>(a, epi, p->stream);
    return launch_zinv<T>(a, epi, p->lds_z, p->stream);
}

void fill_common(mm_plan *p, ZInvArgs &a, unsigned terms, const void *Ms, double Ms_s, double A) {
    std::memset(&a, 0, sizeof a);
    a.g = p->zg;
    a.i32 = p->i32 ? 1 : 0;
    a.terms = terms;
    a.Ms = Ms; a.Ms_scalar = Ms_s;
    a.ex_pref = 2.0 * A / kMu0;
    for (int i = 0; i < 3; ++i) a.inv_d2[i] = 1.0 / (p->d[i] * p->d[i]);
    a.dmi_kind = p->dmi_kind;
    a.dmi_pref = 2.0 * p->dmi_D / kMu0;
    for (int i = 0; i < 3; ++i) a.inv_2d[i] = 0.5 / p->d[i];
    a.ku_pref = 2.0 * p->ku / kMu0;
    for (int i = 0; i < 3; ++i) a.ku_axis[i] = p->ku_axis[i];
    a.stt_pref = p->stt_j != 0.0 ? kHbar * p->stt_j / (kMu0 * kECharge * p->stt_d) : 0.0;
    const double l2 = p->stt_lambda * p->stt_lambda;
    a.stt_pl2 = p->stt_P * l2;
    a.stt_l2p1 = l2 + 1.0;
    a.stt_l2m1 = l2 - 1.0;
    a.stt_epsp = p->stt_epsp;
    for (int i = 0; i < 3; ++i) a.stt_p[i] = p->stt_p[i];
}

int check_plan(mm_plan *p) {
    if (!p) return fail(MM_EINVAL, "plan is NULL");
    if (!p->tensor) return fail(MM_ESTATE, "plan has no tensor (demag_tensor_init or mm_plan_attach_memory did not complete)");
    return MM_OK;
}

int check_material(const void *Ms, double Ms_scalar, double A, unsigned terms) {
    if (!std::isfinite(Ms_scalar) || !std::isfinite(A)) return fail(MM_EINVAL, "Ms_scalar and A must be finite");
    if (!Ms && !(Ms_scalar >= 0.0)) return fail(MM_EINVAL, "Ms_scalar must be >= 0");
    if ((terms & MM_EXCHANGE) && !(A >= 0.0)) return fail(MM_EINVAL, "A must be >= 0");
    return MM_OK;
}

template <typename T>
int heff_impl(mm_plan *p, const void *m, const void *Ms, double Ms_s, double A, void *h, unsigned terms, double *E) {
    int rc;
    if (terms & MM_DEMAG) {
        if ((rc = run_zfwd<T>(p, SRC_MS_M, m, Ms, Ms_s))) return rc;
        if ((rc = run_xyx<T>(p))) return rc;
    }
    ZInvArgs a;
    fill_common(p, a, terms, Ms, Ms_s, A);
    a.m = m; a.h_out = h; a.epart = E ? p->epart : nullptr;
    int nblk = zinv_tiles(p);
    if (!(terms & MM_DEMAG) && ((terms & MM_EXCHANGE) || p->dmi_kind) && p->st_blocks > 0) {
        // no transform, neighbours needed: the stencil kernel streams m once
        // (local terms alone take the z pass's epilogue, which loads no neighbours)
        HIPCK(launch_stencil_heff<T>(a, p->st_cx, p->st_nqb, p->st_blocks, p->stream));
        nblk = p->st_blocks;
    } else {
        HIPCK(zinv_any<T>(p, a, EPI_HEFF));
    }
    if (E) {
        HIPCK(launch_energy_reduce(p->epart, nblk, p->esum, p->stream));
        double s[2];
        HIPCK(hipMemcpyAsync(s, p->esum, sizeof s, hipMemcpyDeviceToHost, p->stream));
        HIPCK(hipStreamSynchronize(p->stream));
        const double V = p->d[0] * p->d[1] * p->d[2];
        E[0] = -0.5 * kMu0 * V * s[0];
        E[1] = -0.5 * kMu0 * V * s[1];
        if (!std::isfinite(E[0]) || !std::isfinite(E[1])) return fail(MM_ENONFINITE, "energies are not finite (E_d=%g, E_ex=%g)", E[0], E[1]);
    }
    return MM_OK;
}

// enqueue one RK4 step (17 launches)
template <typename T>
int enqueue_step(mm_plan *p, void *m, const void *Ms, double Ms_s, double A, double alpha, double gamma, double dt,
                 const double *hext, int renorm) {
    int rc;
    if ((rc = run_zfwd<T>(p, SRC_MS_M, m, Ms, Ms_s))) return rc;
    for (int s = 0; s < 4; ++s) {
        if ((rc = run_xyx<T>(p))) return rc;
        ZInvArgs a;
        fill_common(p, a, MM_DEMAG | MM_EXCHANGE, Ms, Ms_s, A);
        if (hext) for (int i = 0; i < 3; ++i) a.hext[i] = hext[i];
        a.stage = s;
        a.next_r2c = s < 3;
        a.renorm = renorm;
        a.dt = dt; a.alpha = alpha; a.gp = gamma / (1.0 + alpha * alpha);
        a.ms_in = s == 0 ? m : p->ms[(s - 1) & 1];
        a.m_n = m; a.acc = p->acc;
        a.ms_out = s < 3 ? p->ms[s & 1] : nullptr;
        a.m_out = s == 3 ? m : nullptr;
        HIPCK(zinv_any<T>(p, a, EPI_STAGE));
    }
    return MM_OK;
}

template <typename T>
int llg_impl(mm_plan *p, void *m, const void *Ms, double Ms_s, double A, double alpha, double gamma, double dt,
             int n, const double *hext, unsigned flags) {
    const int renorm = (flags & MM_NO_RENORM) ? 0 : 1;
    if (flags & MM_NO_GRAPH) {
        for (int k = 0; k < n; ++k) {
            int rc = enqueue_step<T>(p, m, Ms, Ms_s, A, alpha, gamma, dt, hext, renorm);
            if (rc) return rc;
        }
        return MM_OK;
    }
    // graph key: every argument baked into the captured launches
    std::vector<unsigned char> key(128, 0);
    double vals[10] = {Ms_s, A, alpha, gamma, dt, hext ? hext[0] : 0.0, hext ? hext[1] : 0.0, hext ? hext[2] : 0.0, (double)renorm, hext ? 1.0 : 0.0};
    const void *ptrs[3] = {m, Ms, (const void *)p->stream};
    std::memcpy(key.data(), vals, sizeof vals);
    std::memcpy(key.data() + sizeof vals, ptrs, sizeof ptrs);
    if (!p->gexec || key != p->gkey) {
        if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
        hipGraph_t graph = nullptr;
        if (!p->cap) HIPCK(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
        hipStream_t user = p->stream;
        p->stream = p->cap;
        hipError_t e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) { p->stream = user; return fail(MM_EHIP, "begin capture: %s", hipGetErrorString(e)); }
        int rc = enqueue_step<T>(p, m, Ms, Ms_s, A, alpha, gamma, dt, hext, renorm);
        e = hipStreamEndCapture(p->cap, &graph);
        p->stream = user;
        if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
        if (e != hipSuccess) return fail(MM_EHIP, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) { p->gexec = nullptr; return fail(MM_EHIP, "graph instantiate: %s", hipGetErrorString(e)); }
        p->gkey = key;
    }
    for (int k = 0; k < n; ++k) HIPCK(hipGraphLaunch(p->gexec, p->stream));
    return MM_OK;
}

template <typename T>
int adjoint_impl(mm_plan *p, const void *m, const void *Ms, double Ms_s, double A, const void *g_h, void *g_m,
                 void *g_Ms, unsigned terms, int acc_gMs) {
    int rc;
    if (terms & MM_DEMAG) {
        if ((rc = run_zfwd<T>(p, SRC_RAW, g_h, nullptr, 1.0))) return rc;
        if ((rc = run_xyx<T>(p))) return rc;
    }
    ZInvArgs a;
    fill_common(p, a, terms, Ms, Ms_s, A);
    a.m = m; a.g_h = g_h; a.g_m = g_m; a.g_Ms = g_Ms; a.acc_gMs = acc_gMs;
    HIPCK(zinv_any<T>(p, a, EPI_ADJ));
    return MM_OK;
}

// scratch of the RK4 adjoint: s1..s3, h0..h3, u, ub, kb, ym, yh, gmh (14 vector fields)
template <typename T>
int llg_adjoint_impl(mm_plan *p, const void *m, const void *Ms, double Ms_s, double A, double alpha, double gamma,
                     double dt, const double *hext, unsigned flags, void *g, void *g_Ms, void *fixed_scr = nullptr) {
    const int64_t ncell = p->n[0] * p->n[1] * p->n[2];
    int rc;
    size_t need[3];
    scratch_need(ncell, sizeof(T), zinv_tiles(p), need);
    // the caller's fixed region (checked large enough), else the plan's scratch
    void *scr = fixed_scr;
    if (!scr && (rc = get_scratch(p, need[0], &scr))) return rc;
    T *base = (T *)scr;
    auto buf = [&](int i) { return (void *)(base + (size_t)i * ncell * 3); };
    void *srec[4] = {(void *)m, buf(0), buf(1), buf(2)};
    void *hrec[4] = {buf(3), buf(4), buf(5), buf(6)};
    void *urec = buf(7), *ub = buf(8), *kb = buf(9), *ym = buf(10), *yh = buf(11), *gmh = buf(12);
    const int renorm = (flags & MM_NO_RENORM) ? 0 : 1;
    const double gp = gamma / (1.0 + alpha * alpha);
    // forward recompute with stage records
    if ((rc = run_zfwd<T>(p, SRC_MS_M, m, Ms, Ms_s))) return rc;
    for (int s = 0; s < 4; ++s) {
        if ((rc = run_xyx<T>(p))) return rc;
        ZInvArgs a;
        fill_common(p, a, MM_DEMAG | MM_EXCHANGE, Ms, Ms_s, A);
        if (hext) for (int i = 0; i < 3; ++i) a.hext[i] = hext[i];
        a.stage = s; a.next_r2c = s < 3; a.renorm = renorm;
        a.dt = dt; a.alpha = alpha; a.gp = gp;
        a.ms_in = srec[s]; a.m_n = m; a.acc = p->acc;
        a.ms_out = s < 3 ? srec[s + 1] : nullptr;
        a.m_out = nullptr; a.h_rec = hrec[s]; a.u_rec = s == 3 ? urec : nullptr;
        HIPCK(zinv_any<T>(p, a, EPI_STAGE));
    }
    // reverse
    HIPCK(launch_adj_unorm<T>((const T *)g, (const T *)urec, (T *)ub, (T *)g, renorm, ncell, p->stream));
    const double w[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
    const double coef[4] = {0.0, 0.5 * dt, 0.5 * dt, dt};
    HIPCK(launch_scale_copy<T>((const T *)ub, (T *)kb, w[3], ncell * 3, p->stream));   // kb = (dt/6) u_bar
    for (int q = 3; q >= 0; --q) {
        if ((rc = run_zfwd<T>(p, SRC_ADJPRE, nullptr, nullptr, 1.0, srec[q], hrec[q], kb, ym, yh, gp, alpha))) return rc;
        if ((rc = run_xyx<T>(p))) return rc;
        ZInvArgs a;
        fill_common(p, a, MM_DEMAG | MM_EXCHANGE, Ms, Ms_s, A);
        a.m = srec[q]; a.g_h = yh; a.g_m = gmh; a.g_Ms = g_Ms; a.acc_gMs = 1;
        HIPCK(zinv_any<T>(p, a, EPI_ADJ));
        HIPCK(launch_adj_combine<T>((const T *)ym, (const T *)gmh, (const T *)ub, (T *)g, q > 0 ? (T *)kb : nullptr,
                                    q > 0 ? w[q - 1] : 0.0, coef[q], ncell * 3, p->stream));
    }
    return MM_OK;
}

// Fehlberg's 4(5) pair: stage matrix rows, fourth- and fifth-order weights
const double kRkfA[6][5] = {{0, 0, 0, 0, 0},
                            {1.0 / 4, 0, 0, 0, 0},
                            {3.0 / 32, 9.0 / 32, 0, 0, 0},
                            {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197, 0, 0},
                            {439.0 / 216, -8.0, 3680.0 / 513, -845.0 / 4104, 0},
                            {-8.0 / 27, 2.0, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40}};
const double kRkfB4[6] = {25.0 / 216, 0, 1408.0 / 2565, 2197.0 / 4104, -1.0 / 5, 0};
const double kRkfB5[6] = {16.0 / 135, 0, 6656.0 / 12825, 28561.0 / 56430, -9.0 / 50, 2.0 / 55};

// one attempted RKF45 step: six stages through the demag pipeline, the
// fourth-order candidate in the plan's buffer, the max-norm error on the host
template <typename T>
int rkf45_impl(mm_plan *p, void *m, const void *Ms, double Ms_s, double A, double alpha, double gamma, double dt,
               const double *hext, int renorm, double *err) {
    const size_t f3 = (size_t)p->n[0] * p->n[1] * p->n[2] * 3 * sizeof(T);
    int rc;
    size_t need[3];
    scratch_need(p->n[0] * p->n[1] * p->n[2], sizeof(T), zinv_tiles(p), need);
    void *K = nullptr;
    if ((rc = get_scratch(p, need[1], &K))) return rc;
    void *cand = static_cast<char *>(K) + 6 * f3;
    if ((rc = run_zfwd<T>(p, SRC_MS_M, m, Ms, Ms_s))) return rc;
    for (int s = 0; s < 6; ++s) {
        if ((rc = run_xyx<T>(p))) return rc;
        ZInvArgs a;
        fill_common(p, a, MM_DEMAG | MM_EXCHANGE, Ms, Ms_s, A);
        if (hext) for (int i = 0; i < 3; ++i) a.hext[i] = hext[i];
        a.tab_s = s;
        a.tab_last = s == 5;
        a.next_r2c = s < 5;
        a.renorm = renorm;
        a.dt = dt; a.alpha = alpha; a.gp = gamma / (1.0 + alpha * alpha);
        a.ms_in = s == 0 ? m : p->ms[(s - 1) & 1];
        a.m_n = m;
        a.ms_out = s < 5 ? p->ms[s & 1] : nullptr;
        a.K = K; a.kstride = (int64_t)p->n[0] * p->n[1] * p->n[2] * 3; a.cand = cand;
        for (int j = 0; j <= s; ++j) {
            if (s < 5) a.tab_a[j] = kRkfA[s + 1][j];
            else { a.tab_a[j] = kRkfB4[j]; a.tab_e[j] = kRkfB5[j] - kRkfB4[j]; }
        }
        a.tab_as = a.tab_a[s];
        a.tab_es = a.tab_e[s];
        a.epart = p->epart;
        HIPCK(zinv_any<T>(p, a, EPI_TAB));
    }
    HIPCK(launch_max_reduce(p->epart, zinv_tiles(p), p->esum, p->stream));
    double e = 0.0;
    HIPCK(hipMemcpyAsync(&e, p->esum, sizeof e, hipMemcpyDeviceToHost, p->stream));
    HIPCK(hipStreamSynchronize(p->stream));
    *err = e;
    return MM_OK;
}

// Barzilai-Borwein energy minimisation (synchronous: the host reads the
// global sums and the maximum torque after every gradient evaluation)
template <typename T>
int bb_impl(mm_plan *p, void *m, const void *Ms, double Ms_s, double A, const double *hext, double tol, int max_iter,
            int *iters, double *torque_out) {
    const int64_t ncell = p->n[0] * p->n[1] * p->n[2];
    const size_t f3 = align256((size_t)ncell * 3 * sizeof(T));
    int rc;
    size_t need[3];
    scratch_need(ncell, sizeof(T), zinv_tiles(p), need);
    void *scr = nullptr;
    if ((rc = get_scratch(p, need[2], &scr))) return rc;
    char *base = static_cast<char *>(scr);
    T *mprev = reinterpret_cast<T *>(base);
    T *g[2] = {reinterpret_cast<T *>(base + f3), reinterpret_cast<T *>(base + 2 * f3)};
    double *part = reinterpret_cast<double *>(base + 3 * f3);
    double *tot = reinterpret_cast<double *>(base + 3 * f3 + align256((size_t)zinv_tiles(p) * 4 * sizeof(double)));
    double torque = 0.0;
    int k = 0;
    for (;; ++k) {
        if ((rc = run_zfwd<T>(p, SRC_MS_M, m, Ms, Ms_s))) return rc;
        if ((rc = run_xyx<T>(p))) return rc;
        ZInvArgs a;
        fill_common(p, a, MM_DEMAG | MM_EXCHANGE, Ms, Ms_s, A);
        if (hext) for (int i = 0; i < 3; ++i) a.hext[i] = hext[i];
        a.m = m;
        a.bb_g = g[k & 1];
        a.bb_mprev = mprev;
        a.bb_gprev = g[(k + 1) & 1];
        a.bb_prev = k >= 1;
        a.bb_part = part;
        HIPCK(zinv_any<T>(p, a, EPI_BB));
        HIPCK(launch_bb_reduce(part, zinv_tiles(p), tot, p->stream));
        double s[4];
        HIPCK(hipMemcpyAsync(s, tot, sizeof s, hipMemcpyDeviceToHost, p->stream));
        HIPCK(hipStreamSynchronize(p->stream));
        torque = s[3];
        if (!std::isfinite(torque)) { *iters = k; *torque_out = torque; return fail(MM_ENONFINITE, "torque is not finite"); }
        if (torque <= tol || k >= max_iter) break;
        double tau = 0.0;
        if (k >= 1) tau = (k & 1) ? s[0] / s[1] : s[1] / s[2];
        if (!(std::isfinite(tau) && tau > 0.0)) tau = 0.01 / torque;
        HIPCK(launch_bb_update<T>(static_cast<T *>(m), g[k & 1], mprev, tau, ncell, p->stream));
    }
    *iters = k;
    *torque_out = torque;
    return MM_OK;
}

// one launch of pass k on the plan's scratch arrays (timing only)
template <typename T>
int time_one(mm_plan *p, int k) {
    switch (k) {
    case 0: return run_zfwd<T>(p, SRC_MS_M, p->ms[0], nullptr, 8e5);
    case 1:
        if (p->x_ct) HIPCK(launch_x<T>(p, -1));
        else HIPCK(launch_line_pass<T>(p->d_lp, nullptr, p->tiles_fwd, p->lp_fwd.nthr, p->lds_fwd, -1, false, p->stream));
        return MM_OK;
    case 2:
        if (p->y_ct) HIPCK(launch_y<T>(p));
        else HIPCK(launch_fused_y<T>(p->d_fp, nullptr, p->fp.tiles, p->fp.nthr, p->lds_fp, p->stream));
        return MM_OK;
    case 3:
        if (p->x_ct) HIPCK(launch_x<T>(p, +1));
        else HIPCK(launch_line_pass<T>(p->d_lp + 1, nullptr, p->tiles_inv, p->lp_inv.nthr, p->lds_inv, +1, false, p->stream));
        return MM_OK;
    case 4: {
        ZInvArgs a;
        fill_common(p, a, MM_DEMAG | MM_EXCHANGE, nullptr, 8e5, 1.3e-11);
        a.stage = 1; a.next_r2c = 1; a.renorm = 1; a.dt = 1e-13; a.alpha = 0.02; a.gp = 2.2e5;
        a.ms_in = p->ms[0]; a.m_n = p->ms[0]; a.acc = p->acc; a.ms_out = p->ms[1];
        HIPCK(zinv_any<T>(p, a, EPI_STAGE));
        return MM_OK;
    }
    default: {
        ZInvArgs a;
        fill_common(p, a, MM_DEMAG | MM_EXCHANGE, nullptr, 8e5, 1.3e-11);
        a.m = p->ms[0]; a.h_out = p->ms[1];
        HIPCK(zinv_any<T>(p, a, EPI_HEFF));
        return MM_OK;
    }
    }
}

}  // namespace

// =============================== C ABI ======================================
extern "C" {

int mm_plan_opts_default(mm_plan_opts *o) {
    if (!o) return fail(MM_EINVAL, "opts is NULL");
    std::memset(o, 0, sizeof *o);
    o->far_radius = 16.0;
    o->pow2_padding = 2;
    return MM_OK;
}

}  // extern "C"

namespace {
// argument checks and padded lengths shared by plan creation and sizing
int plan_params(const int64_t grid[3], const double cell[3], int precision, const mm_plan_opts *opts,
                mm_plan_opts *o_out, int64_t L[3]) {
    int rc = validate_grid(grid, cell);
    if (rc) return rc;
    if (precision != MM_F32 && precision != MM_F64) return fail(MM_EINVAL, "precision must be MM_F32 or MM_F64");
    mm_plan_opts o;
    mm_plan_opts_default(&o);
    if (opts) o = *opts;
    if (!std::isfinite(o.far_radius)) return fail(MM_EINVAL, "far_radius must be finite");
    if (o.pow2_padding < 0 || o.pow2_padding > 3) return fail(MM_EINVAL, "pow2_padding must be 0, 1, 2 or 3");
    for (int a = 0; a < 3; ++a) {
        L[a] = o.L[a] > 0 ? o.L[a]
               : o.pow2_padding == 1 ? pow2_L(grid[a])
               : o.pow2_padding == 2 ? auto_L(grid[a], a, precision)
               : o.pow2_padding == 3 ? ct_L(grid[a], a, precision)
                                     : default_L(grid[a]);
        if (L[a] < 2 * grid[a] - 1 || !is_7smooth(L[a]))
            return fail(MM_EINVAL, "L[%d]=%lld must be 7-smooth and >= 2n-1 = %lld", a, (long long)L[a], (long long)(2 * grid[a] - 1));
        if (L[a] > 16384) return fail(MM_ENOTSUP, "L[%d]=%lld exceeds 16384", a, (long long)L[a]);
    }
    if (o.autotune < 0 || o.autotune > 2) return fail(MM_EINVAL, "autotune must be 0 (off), 1 (cached) or 2 (search)");
    const int64_t ncell = grid[0] * grid[1] * grid[2];
    if (grid[0] * grid[1] > 0x7fffffffLL / 2 || ncell > (1LL << 34)) return fail(MM_ENOTSUP, "grid too large");
    *o_out = o;
    return MM_OK;
}
}  // namespace

extern "C" {

int demag_tensor_init(mm_plan **out, const int64_t grid[3], const double cell[3], int precision, void *hip_stream,
                      const mm_plan_opts *opts) {
    if (!out) return fail(MM_EINVAL, "out is NULL");
    *out = nullptr;
    mm_plan_opts o;
    int64_t L[3];
    int rc = plan_params(grid, cell, precision, opts, &o, L);
    if (rc) return rc;
    int dev = 0;
    HIPCK(hipGetDevice(&dev));
    mm_plan *p = new (std::nothrow) mm_plan();
    if (!p) return fail(MM_ENOMEM, "plan allocation");
    p->prec = precision;
    p->rsz = precision == MM_F32 ? 4 : 8;
    p->device = dev;
    p->stream = (hipStream_t)hip_stream;
    p->P = o.far_radius;
    for (int a = 0; a < 3; ++a) { p->n[a] = grid[a]; p->d[a] = cell[a]; p->L[a] = L[a]; }
    rc = precision == MM_F32 ? setup_plan<float>(p, &o) : setup_plan<double>(p, &o);
    // 32-bit indices: 3 values per cell and 3 complex values per (kz, x, y)
    // of S1 below 2^31 (MMX_NO_I32: test hook keeping 64-bit indices)
    {
        const uint64_t cells = (uint64_t)grid[0] * grid[1] * grid[2];
        const uint64_t s1 = (uint64_t)p->hz * grid[0] * grid[1];
        p->i32 = 3 * cells < (uint64_t(1) << 31) && 3 * s1 < (uint64_t(1) << 31) && !getenv("MMX_NO_I32");
    }
    if (!rc) rc = compute_tensor(p);
    const int tm = tune_mode(o.autotune);
    if (!rc && tm) rc = precision == MM_F32 ? autotune_x<float>(p, tm) : autotune_x<double>(p, tm);
    if (!rc && tm) rc = precision == MM_F32 ? autotune_y<float>(p, tm) : autotune_y<double>(p, tm);
    if (!rc && tm) rc = precision == MM_F32 ? autotune_radix<float>(p, tm) : autotune_radix<double>(p, tm);
    if (rc) {
        std::string keep = g_last;
        free_all(p);
        delete p;
        g_last = keep;
        return rc;
    }
    *out = p;
    return MM_OK;
}

int mm_plan_destroy(mm_plan *p) {
    if (!p) return fail(MM_EINVAL, "plan is NULL");
    (void)hipStreamSynchronize(p->stream);
    free_all(p);
    if (p->ev) (void)hipEventDestroy(p->ev);
    delete p;
    return MM_OK;
}

int mm_plan_bytes(const int64_t grid[3], int precision, const mm_plan_opts *opts, size_t *tensor_bytes,
                  size_t *workspace_bytes) {
    if (!tensor_bytes || !workspace_bytes) return fail(MM_EINVAL, "tensor_bytes and workspace_bytes must be non-NULL");
    const double unit[3] = {1.0, 1.0, 1.0};   // sizes do not depend on the cell
    mm_plan_opts o;
    int64_t L[3];
    int rc = plan_params(grid, unit, precision, opts, &o, L);
    if (rc) return rc;
    mm_plan q;
    q.dry = true;
    q.prec = precision;
    q.rsz = precision == MM_F32 ? 4 : 8;
    for (int a = 0; a < 3; ++a) { q.n[a] = grid[a]; q.d[a] = 1.0; q.L[a] = L[a]; }
    rc = precision == MM_F32 ? setup_plan<float>(&q, &o) : setup_plan<double>(&q, &o);
    if (rc) return rc;
    *tensor_bytes = q.tensor_bytes;
    *workspace_bytes = q.ws_used;
    return MM_OK;
}

int mm_plan_attach_memory(mm_plan *p, void *tensor_buf, void *workspace_buf) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!tensor_buf || !workspace_buf) return fail(MM_EINVAL, "tensor_buf and workspace_buf must be non-NULL");
    if (((uintptr_t)tensor_buf | (uintptr_t)workspace_buf) & 255) return fail(MM_EINVAL, "buffers must be 256-byte aligned");
    if (p->ws) return fail(MM_ESTATE, "memory is already attached to this plan");
    HIPCK(hipStreamSynchronize(p->stream));
    // the tensor spectrum moves into the caller's buffer
    HIPCK(hipMemcpy(tensor_buf, p->tensor, p->tensor_bytes, hipMemcpyDeviceToDevice));
    const int xv0 = p->x_var[0], xv1 = p->x_var[1], yv = p->y_var;
    free_all(p);   // the plan's own buffers, captured graph and plan-owned scratch
    p->bytes = 0;
    p->tensor = nullptr;
    p->ws = static_cast<char *>(workspace_buf);
    p->ws_used = 0;
    p->tensor_ext = tensor_buf;
    mm_plan_opts o;
    mm_plan_opts_default(&o);
    rc = p->prec == MM_F32 ? setup_plan<float>(p, &o) : setup_plan<double>(p, &o);
    if (!rc) rc = configure_x(p, 0, xv0);
    if (!rc) rc = configure_x(p, 1, xv1);
    if (rc) { p->tensor = nullptr; return rc; }   // the plan is unusable (MM_ESTATE) from here
    p->y_var = p->y_ct ? yv : 0;
    return MM_OK;
}

int mm_plan_set_dmi(mm_plan *p, int kind, double D) {
    if (!p) return fail(MM_EINVAL, "plan is NULL");
    if (kind < 0 || kind > 2) return fail(MM_EINVAL, "kind must be 0 (none), 1 (interfacial) or 2 (bulk)");
    if (!std::isfinite(D)) return fail(MM_EINVAL, "D must be finite");
    (void)hipStreamSynchronize(p->stream);
    p->dmi_kind = D != 0.0 ? kind : 0;
    p->dmi_D = D;
    // a captured step holds the field arguments by value
    if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
    return MM_OK;
}

int mm_plan_set_anisotropy(mm_plan *p, double Ku, const double axis[3]) {
    if (!p) return fail(MM_EINVAL, "plan is NULL");
    if (!std::isfinite(Ku)) return fail(MM_EINVAL, "Ku must be finite");
    double u[3] = {0.0, 0.0, 1.0};
    if (Ku != 0.0) {
        if (!axis) return fail(MM_EINVAL, "axis must be non-NULL");
        const double nrm = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) return fail(MM_EINVAL, "axis must be finite and non-zero");
        for (int i = 0; i < 3; ++i) u[i] = axis[i] / nrm;
    }
    (void)hipStreamSynchronize(p->stream);
    p->ku = Ku;
    for (int i = 0; i < 3; ++i) p->ku_axis[i] = u[i];
    if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
    return MM_OK;
}

int mm_plan_set_stt(mm_plan *p, double j, double P, double lambda, double eps_prime, double d_layer,
                    const double pol[3]) {
    if (!p) return fail(MM_EINVAL, "plan is NULL");
    if (!std::isfinite(j) || !std::isfinite(P) || !std::isfinite(lambda) || !std::isfinite(eps_prime) ||
        !std::isfinite(d_layer))
        return fail(MM_EINVAL, "spin-transfer parameters must be finite");
    double u[3] = {0.0, 0.0, 1.0};
    if (j != 0.0) {
        if (!(lambda > 0.0)) return fail(MM_EINVAL, "lambda must be > 0");
        if (!(d_layer > 0.0)) return fail(MM_EINVAL, "the free-layer thickness must be > 0");
        if (!pol) return fail(MM_EINVAL, "the polarisation vector must be non-NULL");
        const double nrm = std::sqrt(pol[0] * pol[0] + pol[1] * pol[1] + pol[2] * pol[2]);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) return fail(MM_EINVAL, "the polarisation vector must be finite and non-zero");
        for (int i = 0; i < 3; ++i) u[i] = pol[i] / nrm;
    }
    (void)hipStreamSynchronize(p->stream);
    p->stt_j = j;
    p->stt_P = P; p->stt_lambda = j != 0.0 ? lambda : 1.0; p->stt_epsp = eps_prime;
    p->stt_d = j != 0.0 ? d_layer : 1.0;
    for (int i = 0; i < 3; ++i) p->stt_p[i] = u[i];
    if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
    return MM_OK;
}

int mm_plan_set_stream(mm_plan *p, void *s) {
    if (!p) return fail(MM_EINVAL, "plan is NULL");
    hipStream_t ns = (hipStream_t)s;
    if (ns == p->stream) return MM_OK;
    // the plan's workspace, scratch and graph are shared by every call: the
    // new stream waits for what is already queued on the old one
    if (!p->ev) HIPCK(hipEventCreateWithFlags(&p->ev, hipEventDisableTiming));
    HIPCK(hipEventRecord(p->ev, p->stream));
    HIPCK(hipStreamWaitEvent(ns, p->ev, 0));
    p->stream = ns;
    return MM_OK;
}

int mm_plan_scratch_bytes(const int64_t grid[3], int precision, const mm_plan_opts *opts, size_t bytes_out[3]) {
    if (!bytes_out) return fail(MM_EINVAL, "bytes_out must be non-NULL");
    const double unit[3] = {1.0, 1.0, 1.0};
    mm_plan_opts o;
    int64_t L[3];
    int rc = plan_params(grid, unit, precision, opts, &o, L);
    if (rc) return rc;
    mm_plan q;
    q.dry = true;
    q.prec = precision;
    q.rsz = precision == MM_F32 ? 4 : 8;
    for (int a = 0; a < 3; ++a) { q.n[a] = grid[a]; q.d[a] = 1.0; q.L[a] = L[a]; }
    rc = precision == MM_F32 ? setup_plan<float>(&q, &o) : setup_plan<double>(&q, &o);
    if (rc) return rc;
    scratch_need(grid[0] * grid[1] * grid[2], q.rsz, zinv_tiles(&q), bytes_out);
    return MM_OK;
}

int mm_plan_attach_scratch(mm_plan *p, void *buf, size_t bytes) {
    if (!p) return fail(MM_EINVAL, "plan is NULL");
    if (!buf || bytes == 0) return fail(MM_EINVAL, "buf must be non-NULL and bytes > 0");
    if ((uintptr_t)buf & 255) return fail(MM_EINVAL, "buf must be 256-byte aligned");
    HIPCK(hipStreamSynchronize(p->stream));
    if (p->scr && !p->scr_ext) {
        auto it = std::find(p->allocs.begin(), p->allocs.end(), p->scr);
        if (it != p->allocs.end()) p->allocs.erase(it);
        (void)hipFree(p->scr);
        p->bytes -= p->scr_bytes;
    }
    p->scr = buf;
    p->scr_bytes = bytes;
    p->scr_ext = true;
    return MM_OK;
}

int mm_plan_info(const mm_plan *p, int64_t L[3], size_t *bytes, int tiles[5]) {
    if (!p) return fail(MM_EINVAL, "plan is NULL");
    if (L) for (int a = 0; a < 3; ++a) L[a] = p->L[a];
    if (bytes) *bytes = p->bytes;
    if (tiles) { tiles[0] = p->zg.P; tiles[1] = p->lp_fwd.W; tiles[2] = p->y_ct ? p->y_var : -p->fp.W; tiles[3] = p->x_var[0]; tiles[4] = p->x_var[1]; }
    return MM_OK;
}

// schedule description as JSON text into buf (len bytes, NUL-terminated)
static int put_text(const std::string &t, char *buf, size_t len) {
    if (!buf) return fail(MM_EINVAL, "buf is NULL");
    if (t.size() + 1 > len) return fail(MM_EINVAL, "buffer of %zu bytes too small for %zu", len, t.size() + 1);
    std::memcpy(buf, t.c_str(), t.size() + 1);
    return MM_OK;
}

static std::string plan_schedule_json(const mm_plan *p) {
    char b[512];
    std::string t = "{";
    snprintf(b, sizeof b, "\"L\": [%lld, %lld, %lld], ", (long long)p->L[0], (long long)p->L[1], (long long)p->L[2]);
    t += b;
    snprintf(b, sizeof b, "\"x_fwd\": {\"specialised\": %d, \"variant\": %d, \"W\": %d}, ", p->x_ct ? 1 : 0, p->x_var[0], p->lp_fwd.W);
    t += b;
    snprintf(b, sizeof b, "\"x_inv\": {\"specialised\": %d, \"variant\": %d, \"W\": %d}, ", p->x_ct ? 1 : 0, p->x_var[1], p->lp_inv.W);
    t += b;
    snprintf(b, sizeof b, "\"y_fused\": {\"specialised\": %d, \"variant\": %d, \"pencils_per_tile\": %d}, ", p->y_ct ? 1 : 0, p->y_ct ? p->y_var : -1, p->fp.W);
    t += b;
    snprintf(b, sizeof b, "\"z\": {\"specialised\": %d, \"columns_per_tile\": %d}, ", p->z_ct ? 1 : 0, p->zg.P);
    t += b;
    const HostFft *f[3] = {&p->fx, &p->fy, &p->fz};
    t += "\"radix_order\": {";
    for (int a = 0; a < 3; ++a) {
        std::string o;
        for (int k = 0; k < f[a]->d.nst; ++k) o += (k ? "," : "") + std::to_string(f[a]->d.rad[k]);
        t += std::string(a ? ", " : "") + "\"" + "xyz"[a] + "\": \"" + o + "\"";
    }
    t += "}}";
    return t;
}

int mm_plan_schedule(const mm_plan *p, char *buf, size_t len) {
    if (!p) return fail(MM_EINVAL, "plan is NULL");
    return put_text(plan_schedule_json(p), buf, len);
}

int h_eff(mm_plan *p, const void *m, const void *Ms, double Ms_scalar, double A, void *h_out, unsigned terms,
          double *energy_out) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!m || !h_out) return fail(MM_EINVAL, "m and h_out must be non-NULL");
    if (m == h_out) return fail(MM_EINVAL, "h_out must not alias m");
    if (terms & ~(MM_DEMAG | MM_EXCHANGE)) return fail(MM_EINVAL, "terms must be a subset of MM_DEMAG|MM_EXCHANGE");
    if (terms == 0 && !p->dmi_kind && p->ku == 0.0 && p->stt_j == 0.0)
        return fail(MM_EINVAL, "terms is empty and the plan has no local terms");
    if ((rc = check_material(Ms, Ms_scalar, A, terms))) return rc;
    return p->prec == MM_F32 ? heff_impl<float>(p, m, Ms, Ms_scalar, A, h_out, terms, energy_out)
                             : heff_impl<double>(p, m, Ms, Ms_scalar, A, h_out, terms, energy_out);
}

static int check_llg(double alpha, double gamma, double dt, const double *hext) {
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(MM_EINVAL, "alpha must be finite and >= 0");
    if (!(gamma > 0.0) || !std::isfinite(gamma)) return fail(MM_EINVAL, "gamma must be finite and > 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(MM_EINVAL, "dt must be finite and > 0");
    if (hext) for (int i = 0; i < 3; ++i) if (!std::isfinite(hext[i])) return fail(MM_EINVAL, "h_ext must be finite");
    return MM_OK;
}

int mm_llg_stability(const double cell[3], double Ms_min, double A, double gamma, double dt, double *omega_dt) {
    if (!cell || !omega_dt) return fail(MM_EINVAL, "cell and omega_dt must be non-NULL");
    for (int a = 0; a < 3; ++a)
        if (!(cell[a] > 0.0) || !std::isfinite(cell[a])) return fail(MM_EINVAL, "cell[%d] must be finite and > 0", a);
    if (!(Ms_min > 0.0) || !std::isfinite(Ms_min)) return fail(MM_EINVAL, "Ms_min must be finite and > 0");
    if (!(A >= 0.0) || !std::isfinite(A)) return fail(MM_EINVAL, "A must be finite and >= 0");
    if (!(gamma > 0.0) || !std::isfinite(gamma) || !(dt > 0.0) || !std::isfinite(dt))
        return fail(MM_EINVAL, "gamma and dt must be finite and > 0");
    double lap = 0.0;
    for (int a = 0; a < 3; ++a) lap += 4.0 / (cell[a] * cell[a]);
    *omega_dt = gamma * (2.0 * A / (kMu0 * Ms_min)) * lap * dt;
    return MM_OK;
}

int llg_step(mm_plan *p, void *m, const void *Ms, double Ms_scalar, double A, double alpha, double gamma, double dt,
             int n_steps, const double h_ext[3], unsigned flags) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!m) return fail(MM_EINVAL, "m must be non-NULL");
    if (n_steps < 0) return fail(MM_EINVAL, "n_steps must be >= 0");
    if (flags & ~(MM_NO_RENORM | MM_NO_GRAPH)) return fail(MM_EINVAL, "unknown flags");
    if ((rc = check_material(Ms, Ms_scalar, A, MM_DEMAG | MM_EXCHANGE))) return rc;
    if ((rc = check_llg(alpha, gamma, dt, h_ext))) return rc;
    if (n_steps == 0) return MM_OK;
    return p->prec == MM_F32 ? llg_impl<float>(p, m, Ms, Ms_scalar, A, alpha, gamma, dt, n_steps, h_ext, flags)
                             : llg_impl<double>(p, m, Ms, Ms_scalar, A, alpha, gamma, dt, n_steps, h_ext, flags);
}

int h_eff_adjoint(mm_plan *p, const void *m, const void *Ms, double Ms_scalar, double A, const void *g_h, void *g_m,
                  void *g_Ms, unsigned terms) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!m || !g_h || !g_m) return fail(MM_EINVAL, "m, g_h and g_m must be non-NULL");
    if (p->dmi_kind || p->ku != 0.0 || p->stt_j != 0.0)
        return fail(MM_ENOTSUP, "the adjoint does not include the DMI, anisotropy or spin-transfer terms");
    if (g_m == g_h || g_m == m) return fail(MM_EINVAL, "g_m must not alias m or g_h");
    if (terms == 0 || (terms & ~(MM_DEMAG | MM_EXCHANGE))) return fail(MM_EINVAL, "terms must be a non-empty subset of MM_DEMAG|MM_EXCHANGE");
    if ((rc = check_material(Ms, Ms_scalar, A, terms))) return rc;
    return p->prec == MM_F32 ? adjoint_impl<float>(p, m, Ms, Ms_scalar, A, g_h, g_m, g_Ms, terms, 0)
                             : adjoint_impl<double>(p, m, Ms, Ms_scalar, A, g_h, g_m, g_Ms, terms, 0);
}

int llg_step_adjoint(mm_plan *p, const void *m, const void *Ms, double Ms_scalar, double A, double alpha, double gamma,
                     double dt, const double h_ext[3], unsigned flags, void *g, void *g_Ms) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!m || !g) return fail(MM_EINVAL, "m and g must be non-NULL");
    if (p->dmi_kind || p->ku != 0.0 || p->stt_j != 0.0)
        return fail(MM_ENOTSUP, "the adjoint does not include the DMI, anisotropy or spin-transfer terms");
    if (g == m) return fail(MM_EINVAL, "g must not alias m");
    if (flags & ~(MM_NO_RENORM | MM_NO_GRAPH)) return fail(MM_EINVAL, "unknown flags");
    if ((rc = check_material(Ms, Ms_scalar, A, MM_DEMAG | MM_EXCHANGE))) return rc;
    if ((rc = check_llg(alpha, gamma, dt, h_ext))) return rc;
    return p->prec == MM_F32 ? llg_adjoint_impl<float>(p, m, Ms, Ms_scalar, A, alpha, gamma, dt, h_ext, flags, g, g_Ms)
                             : llg_adjoint_impl<double>(p, m, Ms, Ms_scalar, A, alpha, gamma, dt, h_ext, flags, g, g_Ms);
}

int llg_step_adjoint_noalloc(mm_plan *p, const void *m, const void *Ms, double Ms_scalar, double A, double alpha,
                             double gamma, double dt, const double h_ext[3], unsigned flags, void *g, void *g_Ms) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!m || !g) return fail(MM_EINVAL, "m and g must be non-NULL");
    if (p->dmi_kind || p->ku != 0.0 || p->stt_j != 0.0)
        return fail(MM_ENOTSUP, "the adjoint does not include the DMI, anisotropy or spin-transfer terms");
    if (g == m) return fail(MM_EINVAL, "g must not alias m");
    if (flags & ~(MM_NO_RENORM | MM_NO_GRAPH)) return fail(MM_EINVAL, "unknown flags");
    if ((rc = check_material(Ms, Ms_scalar, A, MM_DEMAG | MM_EXCHANGE))) return rc;
    if ((rc = check_llg(alpha, gamma, dt, h_ext))) return rc;
    size_t need[3];
    scratch_need(p->n[0] * p->n[1] * p->n[2], p->rsz, zinv_tiles(p), need);
    if (need[0] > (size_t)MM_NOALLOC_SCRATCH_BYTES)
        return fail(MM_ENOTSUP, "llg_step_adjoint_noalloc needs %zu bytes of fixed scratch for this grid; the "
                                "library holds %zu (use llg_step_adjoint)", need[0], (size_t)MM_NOALLOC_SCRATCH_BYTES);
    void *fixed = nullptr;
    hipError_t e = noalloc_scratch(p->device, &fixed);
    if (e != hipSuccess) return fail(MM_EHIP, "fixed scratch address: %s", hipGetErrorString(e));
    return p->prec == MM_F32
               ? llg_adjoint_impl<float>(p, m, Ms, Ms_scalar, A, alpha, gamma, dt, h_ext, flags, g, g_Ms, fixed)
               : llg_adjoint_impl<double>(p, m, Ms, Ms_scalar, A, alpha, gamma, dt, h_ext, flags, g, g_Ms, fixed);
}

int llg_rkf45_step(mm_plan *p, void *m, const void *Ms, double Ms_scalar, double A, double alpha, double gamma,
                   double *dt, double tol, const double h_ext[3], unsigned flags, double *err_out, int *accepted) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!m) return fail(MM_EINVAL, "m must be non-NULL");
    if (!dt || !err_out || !accepted) return fail(MM_EINVAL, "dt, err_out and accepted must be non-NULL");
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(MM_EINVAL, "tol must be finite and > 0");
    if (flags & ~MM_NO_RENORM) return fail(MM_EINVAL, "unknown flags (RKF45 takes MM_NO_RENORM only)");
    if ((rc = check_material(Ms, Ms_scalar, A, MM_DEMAG | MM_EXCHANGE))) return rc;
    if ((rc = check_llg(alpha, gamma, *dt, h_ext))) return rc;
    double err = 0.0;
    rc = p->prec == MM_F32 ? rkf45_impl<float>(p, m, Ms, Ms_scalar, A, alpha, gamma, *dt, h_ext,
                                                (flags & MM_NO_RENORM) ? 0 : 1, &err)
                           : rkf45_impl<double>(p, m, Ms, Ms_scalar, A, alpha, gamma, *dt, h_ext,
                                                 (flags & MM_NO_RENORM) ? 0 : 1, &err);
    if (rc) return rc;
    *err_out = err;
    *accepted = 0;
    if (!std::isfinite(err)) return fail(MM_ENONFINITE, "RKF45 error estimate is not finite");
    if (err <= tol) {
        const size_t f3 = (size_t)p->n[0] * p->n[1] * p->n[2] * 3 * p->rsz;
        HIPCK(hipMemcpyAsync(m, static_cast<char *>(p->scr) + 6 * f3, f3, hipMemcpyDeviceToDevice, p->stream));
        *accepted = 1;
    }
    const double fac = err == 0.0 ? 5.0 : std::min(5.0, std::max(0.2, 0.9 * std::pow(tol / err, 0.2)));
    *dt *= fac;
    return MM_OK;
}

int mm_minimize_bb(mm_plan *p, void *m, const void *Ms, double Ms_scalar, double A, const double h_ext[3],
                   double tol, int max_iter, int *iters_out, double *torque_out) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!m || !iters_out || !torque_out) return fail(MM_EINVAL, "m, iters_out and torque_out must be non-NULL");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(MM_EINVAL, "tol must be finite and >= 0");
    if (max_iter < 0) return fail(MM_EINVAL, "max_iter must be >= 0");
    if ((rc = check_material(Ms, Ms_scalar, A, MM_DEMAG | MM_EXCHANGE))) return rc;
    if (h_ext) for (int i = 0; i < 3; ++i) if (!std::isfinite(h_ext[i])) return fail(MM_EINVAL, "h_ext must be finite");
    return p->prec == MM_F32 ? bb_impl<float>(p, m, Ms, Ms_scalar, A, h_ext, tol, max_iter, iters_out, torque_out)
                             : bb_impl<double>(p, m, Ms, Ms_scalar, A, h_ext, tol, max_iter, iters_out, torque_out);
}

int mm_demag_tensor_get(mm_plan *p, double *host) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!host) return fail(MM_EINVAL, "host_octant is NULL");
    const size_t bytes = (size_t)p->n[0] * p->n[1] * p->n[2] * 6 * sizeof(double);
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) return fail(MM_ENOMEM, "octant: %s", hipGetErrorString(e));
    e = launch_tensor_octant((double *)d, (int)p->n[0], (int)p->n[1], (int)p->n[2], p->d[0], p->d[1], p->d[2], p->P, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host, d, bytes, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(MM_EHIP, "tensor get: %s", hipGetErrorString(e));
    return MM_OK;
}

int mm_demag_tensor_set(mm_plan *p, const double *host) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!host) return fail(MM_EINVAL, "host_octant is NULL");
    const size_t bytes = (size_t)p->n[0] * p->n[1] * p->n[2] * 6 * sizeof(double);
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) return fail(MM_ENOMEM, "octant: %s", hipGetErrorString(e));
    e = hipMemcpyAsync(d, host, bytes, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) { (void)hipFree(d); return fail(MM_EHIP, "tensor set: %s", hipGetErrorString(e)); }
    rc = p->prec == MM_F32 ? build_spectrum<float>(p, (double *)d) : build_spectrum<double>(p, (double *)d);
    (void)hipFree(d);
    return rc;
}

int mm_demag_spectrum_get(mm_plan *p, double *host) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (!host) return fail(MM_EINVAL, "host_spectrum is NULL");
    const size_t bytes = (size_t)p->hx * p->hy * p->hz * 6 * sizeof(double);
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) return fail(MM_ENOMEM, "spectrum: %s", hipGetErrorString(e));
    e = p->prec == MM_F32 ? launch_tensor_export<float>((const float *)p->tensor, (double *)d, p->hx, p->hy, p->hz, p->stream)
                          : launch_tensor_export<double>((const double *)p->tensor, (double *)d, p->hx, p->hy, p->hz, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host, d, bytes, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(MM_EHIP, "spectrum get: %s", hipGetErrorString(e));
    return MM_OK;
}

int mm_plan_time_passes(mm_plan *p, int reps, double *ms) {
    int rc = check_plan(p);
    if (rc) return rc;
    if (reps < 1 || !ms) return fail(MM_EINVAL, "reps must be >= 1 and ms_out non-NULL");
    hipEvent_t e0, e1;
    HIPCK(hipEventCreate(&e0));
    HIPCK(hipEventCreate(&e1));
    for (int k = 0; k < 6 && !rc; ++k) {
        for (int pass = 0; pass < 2 && !rc; ++pass) {   // first round warms up
            const int n = pass == 0 ? 1 : reps;
            (void)hipEventRecord(e0, p->stream);
            for (int r = 0; r < n && !rc; ++r) {
                if (p->prec == MM_F32) rc = time_one<float>(p, k);
                else rc = time_one<double>(p, k);
            }
            (void)hipEventRecord(e1, p->stream);
            hipError_t e = hipEventSynchronize(e1);
            if (e != hipSuccess) rc = fail(MM_EHIP, "time passes: %s", hipGetErrorString(e));
            float t = 0.f;
            (void)hipEventElapsedTime(&t, e0, e1);
            ms[k] = (double)t / n;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int mm_device_copy(void *dst, const void *src, size_t bytes, void *stream) {
    if (!dst || !src || bytes % 16) return fail(MM_EINVAL, "dst/src non-NULL and bytes a multiple of 16");
    HIPCK(launch_copy16(src, dst, (int64_t)(bytes / 16), (hipStream_t)stream));
    return MM_OK;
}

const char *mm_strerror(int s) {
    switch (s) {
    case MM_OK: return "ok";
    case MM_EINVAL: return "invalid argument";
    case MM_ENOMEM: return "out of memory";
    case MM_EHIP: return "HIP runtime error";
    case MM_ESTATE: return "invalid plan state";
    case MM_ENOTSUP: return "not supported";
    case MM_ENONFINITE: return "non-finite result";
    default: return "unknown status";
    }
}

const char *mm_last_error(void) { return g_last.c_str(); }

}  // extern "C"

// =============================== batch ======================================
// A launch group: geometries sharing one kernel for a pass (a specialised
// power-of-two length, or the runtime-planned kernel for everything else).
struct BGroup {
    int L = 0;            // transform length of the group (specialised), 0 = runtime-planned
    int W = 0;            // tile width of the specialised x pass
    int tiles = 0;
    int nthr = 64;
    size_t lds = 0;
    int2 *map = nullptr;  // device tile map (geometry, local tile)
    size_t cap = 0;       // entries the map buffer holds
    int var = 0;          // kernel variant (x: 0..3, y: 0..2, as mm_plan_info)
    std::vector<int> geo; // geometries of the group
};

struct mm_batch {
    int count = 0;
    int prec = MM_F32;
    hipStream_t stream = nullptr;
    std::vector<mm_plan *> plans;
    std::vector<void *> allocs;
    size_t bytes = 0;
    std::vector<BGroup> gxf, gxi, gy, gz;   // forward x, inverse x, fused y, z launch groups
    LinePass *d_lpf = nullptr, *d_lpi = nullptr;
    FusedPass *d_fp = nullptr;
    ZFwdArgs *d_zf = nullptr;
    ZInvArgs *d_zi = nullptr;   // [5][count]: h_eff, stage 0..3
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<unsigned char> gkey, akey;
    // the launch groups of one pass run side by side: up to kSide more
    // streams, forked from and joined back to `stream` by events
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {};
    bool fanout = true;
};

namespace {

int balloc(mm_batch *b, void **out, size_t bytes) {
    *out = nullptr;
    hipError_t e = hipMalloc(out, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) { *out = nullptr; (void)hipGetLastError(); return fail(MM_ENOMEM, "batch hipMalloc(%zu): %s", bytes, hipGetErrorString(e)); }
    b->allocs.push_back(*out);
    b->bytes += bytes;
    return MM_OK;
}

void batch_free(mm_batch *b) {
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    if (b->cap) { (void)hipStreamDestroy(b->cap); b->cap = nullptr; }
    for (int k = 0; k < mm_batch::kSide; ++k) {
        if (b->side[k]) { (void)hipStreamDestroy(b->side[k]); b->side[k] = nullptr; }
        if (b->join[k]) { (void)hipEventDestroy(b->join[k]); b->join[k] = nullptr; }
    }
    if (b->fork) { (void)hipEventDestroy(b->fork); b->fork = nullptr; }
    for (void *q : b->allocs) (void)hipFree(q);
    b->allocs.clear();
    for (mm_plan *p : b->plans) if (p) { free_all(p); delete p; }
    b->plans.clear();
}

// upload the per-call z-pass arguments of every geometry
int batch_args(mm_batch *b, void *const *m_ptrs, const double *Ms, double A, double alpha, double gamma, double dt,
               void *const *h_ptrs, unsigned terms, int renorm) {
    const int n = b->count;
    std::vector<ZFwdArgs> zf(n);
    std::vector<ZInvArgs> zi(5 * (size_t)n);
    for (int g = 0; g < n; ++g) {
        mm_plan *p = b->plans[g];
        std::memset(&zf[g], 0, sizeof(ZFwdArgs));
        zf[g].g = p->zg; zf[g].src = m_ptrs[g]; zf[g].Ms = nullptr; zf[g].Ms_scalar = Ms[g];
        ZInvArgs &h = zi[g];
        fill_common(p, h, terms, nullptr, Ms[g], A);
        h.m = m_ptrs[g]; h.h_out = h_ptrs ? h_ptrs[g] : nullptr;
        for (int s = 0; s < 4; ++s) {
            ZInvArgs &a = zi[(size_t)(1 + s) * n + g];
            fill_common(p, a, MM_DEMAG | MM_EXCHANGE, nullptr, Ms[g], A);
            a.stage = s; a.next_r2c = s < 3; a.renorm = renorm;
            a.dt = dt; a.alpha = alpha; a.gp = gamma / (1.0 + alpha * alpha);
            a.ms_in = s == 0 ? m_ptrs[g] : p->ms[(s - 1) & 1];
            a.m_n = m_ptrs[g]; a.acc = p->acc;
            a.ms_out = s < 3 ? p->ms[s & 1] : nullptr;
            a.m_out = s == 3 ? m_ptrs[g] : nullptr;
        }
    }
    HIPCK(hipMemcpyAsync(b->d_zf, zf.data(), zf.size() * sizeof(ZFwdArgs), hipMemcpyHostToDevice, b->stream));
    HIPCK(hipMemcpyAsync(b->d_zi, zi.data(), zi.size() * sizeof(ZInvArgs), hipMemcpyHostToDevice, b->stream));
    HIPCK(hipStreamSynchronize(b->stream));
    return MM_OK;
}

// Launch the groups of one pass.  With fan-out, the groups (which touch
// disjoint geometries) are spread over `stream` and up to kSide side streams,
// the heaviest first onto the least loaded stream (tiles as the measure of
// work), after an event that forks the side streams from `stream`, and
// `stream` waits for every side stream's join event before the next pass; in
// a captured graph this makes them parallel branches.
template <class F>
int batch_pass(mm_batch *b, const std::vector<BGroup> &gs, const F &launch) {
    int ng = 0;
    for (const BGroup &g : gs) ng += g.tiles > 0;
    if (!b->fanout || ng < 2) {
        for (const BGroup &g : gs) HIPCK(launch(g, b->stream));
        return MM_OK;
    }
    if (!b->fork) {
        HIPCK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        for (int k = 0; k < mm_batch::kSide; ++k) {
            HIPCK(hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking));
            HIPCK(hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming));
        }
    }
    const int nl = std::min(ng, 1 + mm_batch::kSide);
    std::vector<int> order;
    for (int i = 0; i < (int)gs.size(); ++i)
        if (gs[i].tiles > 0) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return gs[x].tiles > gs[y].tiles; });
    std::vector<long long> load(nl, 0);
    std::vector<int> lane(gs.size(), 0);
    for (int i : order) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lane[i] = l;
        load[l] += gs[i].tiles;
    }
    HIPCK(hipEventRecord(b->fork, b->stream));
    for (int l = 1; l < nl; ++l) HIPCK(hipStreamWaitEvent(b->side[l - 1], b->fork, 0));
    for (int i : order) HIPCK(launch(gs[i], lane[i] ? b->side[lane[i] - 1] : b->stream));
    for (int l = 1; l < nl; ++l) {
        HIPCK(hipEventRecord(b->join[l - 1], b->side[l - 1]));
        HIPCK(hipStreamWaitEvent(b->stream, b->join[l - 1], 0));
    }
    return MM_OK;
}

template <typename T>
int batch_zfwd(mm_batch *b) {
    return batch_pass(b, b->gz, [&](const BGroup &g, hipStream_t s) {
        if (g.L) return launch_zfwd_ct_b<T>(b->d_zf, g.map, g.tiles, g.L, SRC_MS_M, s);
        return launch_zfwd_batch<T>(b->d_zf, g.map, g.tiles, g.nthr, SRC_MS_M, g.lds, s);
    });
}

template <typename T>
int batch_zinv(mm_batch *b, const ZInvArgs *d, int epi) {
    return batch_pass(b, b->gz, [&](const BGroup &g, hipStream_t s) {
        if (g.L) return launch_zinv_ct_b<T>(d, g.map, g.tiles, g.L, epi, s);
        return launch_zinv_batch<T>(d, g.map, g.tiles, g.nthr, epi, g.lds, s);
    });
}

template <typename T>
hipError_t batch_x_group(mm_batch *b, const BGroup &g, int dir, hipStream_t s) {
    const LinePass *d = dir < 0 ? b->d_lpf : b->d_lpi;
    if (g.L) return launch_line_var_b<T>(d, g.map, g.tiles, g.L, g.W, dir, g.var, s);
    return launch_line_pass<T>(d, g.map, g.tiles, g.nthr, g.lds, dir, false, s);
}

template <typename T>
hipError_t batch_y_group(mm_batch *b, const BGroup &g, hipStream_t s) {
    if (g.L) return launch_fused_var_b<T>(b->d_fp, g.map, g.tiles, g.L, g.var, s);
    return launch_fused_y<T>(b->d_fp, g.map, g.tiles, g.nthr, g.lds, s);
}

template <typename T>
int batch_xyx(mm_batch *b) {
    int rc;
    if ((rc = batch_pass(b, b->gxf, [&](const BGroup &g, hipStream_t s) { return batch_x_group<T>(b, g, -1, s); })))
        return rc;
    if ((rc = batch_pass(b, b->gy, [&](const BGroup &g, hipStream_t s) { return batch_y_group<T>(b, g, s); })))
        return rc;
    return batch_pass(b, b->gxi, [&](const BGroup &g, hipStream_t s) { return batch_x_group<T>(b, g, +1, s); });
}

template <typename T>
int batch_step(mm_batch *b) {
    int rc;
    if ((rc = batch_zfwd<T>(b))) return rc;
    for (int s = 0; s < 4; ++s) {
        if ((rc = batch_xyx<T>(b))) return rc;
        if ((rc = batch_zinv<T>(b, b->d_zi + (size_t)(1 + s) * b->count, EPI_STAGE))) return rc;
    }
    return MM_OK;
}

template <typename T>
int batch_heff(mm_batch *b, unsigned terms) {
    int rc;
    if (terms & MM_DEMAG) {
        if ((rc = batch_zfwd<T>(b))) return rc;
        if ((rc = batch_xyx<T>(b))) return rc;
    }
    return batch_zinv<T>(b, b->d_zi, EPI_HEFF);
}

std::vector<unsigned char> batch_key(mm_batch *b, void *const *m_ptrs, const double *Ms, double A, double alpha,
                                     double gamma, double dt, void *const *h_ptrs, unsigned terms, int renorm) {
    std::vector<unsigned char> k;
    auto put = [&](const void *p, size_t n) { const unsigned char *c = (const unsigned char *)p; k.insert(k.end(), c, c + n); };
    put(m_ptrs, sizeof(void *) * b->count);
    if (h_ptrs) put(h_ptrs, sizeof(void *) * b->count);
    put(Ms, sizeof(double) * b->count);
    double v[4] = {A, alpha, gamma, dt};
    put(v, sizeof v);
    put(&terms, sizeof terms);
    put(&renorm, sizeof renorm);
    put(&b->stream, sizeof b->stream);
    return k;
}

// (Re)write a group's tile map from its geometries' current tile counts.
template <class Tiles>
int upload_map(BGroup &g, Tiles tiles) {
    std::vector<int2> m;
    for (int i : g.geo) {
        const int t = tiles(i);
        for (int j = 0; j < t; ++j) m.push_back(make_int2(i, j));
    }
    if (m.size() > g.cap) return fail(MM_EINVAL, "tile map of %zu entries exceeds its buffer (%zu)", m.size(), g.cap);
    g.tiles = (int)m.size();
    if (!m.empty()) HIPCK(hipMemcpy(g.map, m.data(), m.size() * sizeof(int2), hipMemcpyHostToDevice));
    return MM_OK;
}

// Build the launch groups of one pass kind: key(plan) = specialised length or
// 0; the map buffer holds `cap_tiles(plan)` tiles per geometry (the most any
// variant the tuner may pick needs).
template <class Key, class Tiles, class Shape, class Cap>
int build_groups(mm_batch *b, std::vector<BGroup> &out, Key key, Tiles tiles, Shape shape, Cap cap_tiles) {
    std::vector<int> keys;
    for (mm_plan *p : b->plans) {
        const int k = key(p);
        if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
    }
    for (int k : keys) {
        BGroup g;
        g.L = k;
        size_t cap = 0;
        for (int i = 0; i < b->count; ++i) {
            mm_plan *p = b->plans[i];
            if (key(p) != k) continue;
            g.geo.push_back(i);
            cap += (size_t)std::max(tiles(p), cap_tiles(p));
            shape(p, g);
        }
        int rc = balloc(b, (void **)&g.map, cap * sizeof(int2));
        if (rc) return rc;
        g.cap = cap;
        if ((rc = upload_map(g, [&](int i) { return tiles(b->plans[i]); }))) return rc;
        out.push_back(std::move(g));
    }
    return MM_OK;
}

// x pass tiles of a plan at the narrowest tile width any variant uses
int x_tiles_max(const mm_plan *p) {
    int t = p->tiles_fwd;
    const size_t csz = p->prec == MM_F32 ? sizeof(float2) : sizeof(double2);
    for (int v : x_variants(p)) {
        int W = 0, NT = 0;
        if (line_ct_shape((int)p->L[0], csz, v, &W, &NT)) t = std::max(t, ((p->lp_fwd.inner + W - 1) / W) * p->lp_fwd.outer);
    }
    return t;
}

// Batch autotuner: per launch group, time every kernel variant the group's
// length has on the batch's own buffers (tile maps rebuilt for each tile
// width) and keep the fastest; winners go to the schedule cache.
template <typename T>
int batch_autotune(mm_batch *b, int mode) {
    if (mode == TUNE_OFF || b->plans.empty()) return MM_OK;
    const int dev = b->plans[0]->device;
    EventPair ev;
    int rc = ev.make();
    for (int d = 0; d < 2 && !rc; ++d) {
        std::vector<BGroup> &gs = d == 0 ? b->gxf : b->gxi;
        LinePass *dd = d == 0 ? b->d_lpf : b->d_lpi;
        for (BGroup &g : gs) {
            if (rc || !g.L) continue;
            mm_plan *p0 = b->plans[g.geo[0]];
            const std::vector<int> cand = x_variants(p0);
            if (cand.size() < 2) continue;
            long long pts = 0;
            for (int i : g.geo) pts += (long long)b->plans[i]->hz * b->plans[i]->n[1] * 3 * g.L;
            const std::string key = tune_key(dev, b->prec, d == 0 ? "batch_x_fwd" : "batch_x_inv", g.L, pts);
            auto apply = [&](int v) -> int {
                for (int i : g.geo) {
                    int r = configure_x(b->plans[i], d, v);
                    if (r) return r;
                    const LinePass &lp = d == 0 ? b->plans[i]->lp_fwd : b->plans[i]->lp_inv;
                    HIPCK(hipMemcpy(dd + i, &lp, sizeof(LinePass), hipMemcpyHostToDevice));
                }
                mm_plan *q = b->plans[g.geo[0]];
                g.var = v;
                g.W = (d == 0 ? q->lp_fwd : q->lp_inv).W;
                return upload_map(g, [&](int i) { return d == 0 ? b->plans[i]->tiles_fwd : b->plans[i]->tiles_inv; });
            };
            std::string got;
            if (mode == TUNE_CACHED && tune_get(key, got)) {
                const int v = atoi(got.c_str());
                if (std::find(cand.begin(), cand.end(), v) != cand.end()) { rc = apply(v); continue; }
            }
            float best = 1e30f;
            int bestv = g.var;
            for (int v : cand) {
                if ((rc = apply(v))) break;
                float ms = 0.f;
                if ((rc = time3(b->stream, ev.a, ev.b, [&] { return batch_x_group<T>(b, g, d == 0 ? -1 : +1, b->stream); }, &ms))) break;
                if (ms < best) { best = ms; bestv = v; }
            }
            if (!rc) rc = apply(bestv);
            if (!rc) tune_put(key, std::to_string(bestv));
        }
    }
    for (BGroup &g : b->gy) {
        if (rc || !g.L) continue;
        std::vector<int> cand{0};
        if (fused_hx_threads(g.L) > 0) cand.push_back(1);
        if (fused_pf_available(g.L, 2)) cand.push_back(2);
        if (cand.size() < 2) continue;
        long long pts = 0;
        for (int i : g.geo) pts += (long long)b->plans[i]->fp.npos * g.L;
        const std::string key = tune_key(dev, b->prec, "batch_y_fused", g.L, pts);
        std::string got;
        if (mode == TUNE_CACHED && tune_get(key, got)) {
            const int v = atoi(got.c_str());
            if (std::find(cand.begin(), cand.end(), v) != cand.end()) { g.var = v; continue; }
        }
        float best = 1e30f;
        int bestv = g.var;
        for (int v : cand) {
            g.var = v;
            float ms = 0.f;
            if ((rc = time3(b->stream, ev.a, ev.b, [&] { return batch_y_group<T>(b, g, b->stream); }, &ms))) break;
            if (ms < best) { best = ms; bestv = v; }
        }
        g.var = bestv;
        if (!rc) tune_put(key, std::to_string(bestv));
    }
    for (BGroup &g : b->gy)
        for (int i : g.geo) b->plans[i]->y_var = g.L ? g.var : 0;
    return rc;
}

}  // namespace

extern "C" {

int mm_batch_create(mm_batch **out, int count, const int64_t (*grids)[3], const double (*cells)[3], int precision,
                    void *hip_stream, const mm_plan_opts *opts) {
    if (!out) return fail(MM_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || count > 65536) return fail(MM_EINVAL, "count must be in [1, 65536]");
    if (!grids || !cells) return fail(MM_EINVAL, "grids and cells must be non-NULL");
    if (precision != MM_F32 && precision != MM_F64) return fail(MM_EINVAL, "precision must be MM_F32 or MM_F64");
    for (int g = 0; g < count; ++g) {
        int rc = validate_grid(grids[g], cells[g]);
        if (rc) return fail(rc, "geometry %d: %s", g, std::string(g_last).c_str());
    }
    mm_plan_opts o;
    mm_plan_opts_default(&o);
    o.pow2_padding = 1;
    if (opts) o = *opts;
    mm_batch *b = new (std::nothrow) mm_batch();
    if (!b) return fail(MM_ENOMEM, "batch allocation");
    b->count = count; b->prec = precision; b->stream = (hipStream_t)hip_stream;
    b->fanout = !getenv("MMX_NO_FANOUT");
    int rc = MM_OK;
    for (int g = 0; g < count && !rc; ++g) {
        mm_plan *p = nullptr;
        mm_plan_opts og = o;
        og.autotune = 0;   // the batch tunes its grouped launches itself
        rc = demag_tensor_init(&p, grids[g], cells[g], precision, hip_stream, &og);
        if (!rc) b->plans.push_back(p);
        // one tile map serves the grouped z-forward and z-inverse launches:
        // linear z tiles for both
        if (!rc) p->zg.ygrp = 0;
        // default grouped x launches (the tuner may change them): the
        // half-LDS kernel on wide tiles for lines of 1024 points or more, the
        // narrow full-LDS kernel below; the MMX_XVAR / MMX_YVAR test hooks
        // keep the variants they set
        if (!rc && !getenv("MMX_XVAR")) {
            int W = 0, NT = 0;
            const size_t csz = precision == MM_F32 ? sizeof(float2) : sizeof(double2);
            const int v = p->x_ct && line_ct_shape((int)p->L[0], csz, 3, &W, &NT) &&
                                  line_hx_lds((int)p->L[0], W, csz) <= kLdsMax ? 3 : 0;
            if (p->x_var[0] != v || p->x_var[1] != v) rc = configure_x(p, v);
        }
        // grouped y launches have variants 0..2, with the whole pencil in LDS
        if (!rc && p->y_ct && fused_ct_lds((int)p->L[1], 2 * p->rsz) > kLdsMax)
            rc = fail(MM_ENOTSUP, "y length %d: no grouped kernel holds its pencil", (int)p->L[1]);
        if (!rc && (!getenv("MMX_YVAR") || p->y_var > 2)) p->y_var = 0;
    }
    std::vector<LinePass> lf, li;
    std::vector<FusedPass> fp;
    for (int g = 0; g < count && !rc; ++g) {
        lf.push_back(b->plans[g]->lp_fwd); li.push_back(b->plans[g]->lp_inv); fp.push_back(b->plans[g]->fp);
    }
    auto xkey = [](mm_plan *p) { return p->x_ct ? (int)p->L[0] : 0; };
    if (!rc) rc = build_groups(b, b->gxf, xkey, [](mm_plan *p) { return p->tiles_fwd; },
                               [](mm_plan *p, BGroup &g) { g.W = p->lp_fwd.W; g.var = p->x_var[0]; g.nthr = std::max(g.nthr, p->lp_fwd.nthr); g.lds = std::max(g.lds, p->lds_fwd); },
                               [](mm_plan *p) { return x_tiles_max(p); });
    if (!rc) rc = build_groups(b, b->gxi, xkey, [](mm_plan *p) { return p->tiles_inv; },
                               [](mm_plan *p, BGroup &g) { g.W = p->lp_inv.W; g.var = p->x_var[1]; g.nthr = std::max(g.nthr, p->lp_inv.nthr); g.lds = std::max(g.lds, p->lds_inv); },
                               [](mm_plan *p) { return x_tiles_max(p); });
    if (!rc) rc = build_groups(b, b->gy, [](mm_plan *p) { return p->y_ct ? (int)p->L[1] : 0; },
                               [](mm_plan *p) { return p->fp.tiles; },
                               [](mm_plan *p, BGroup &g) { g.var = p->y_ct ? p->y_var : 0; g.nthr = std::max(g.nthr, p->fp.nthr); g.lds = std::max(g.lds, p->lds_fp); },
                               [](mm_plan *p) { return p->fp.tiles; });
    if (!rc) rc = build_groups(b, b->gz, [](mm_plan *p) { return p->z_ct ? (int)p->L[2] : 0; },
                               [](mm_plan *p) { return p->zg.tiles; },
                               [](mm_plan *p, BGroup &g) { g.nthr = std::max(g.nthr, p->zg.nthr); g.lds = std::max(g.lds, p->lds_z); },
                               [](mm_plan *p) { return p->zg.tiles; });
    if (!rc) rc = balloc(b, (void **)&b->d_lpf, lf.size() * sizeof(LinePass));
    if (!rc) rc = balloc(b, (void **)&b->d_lpi, li.size() * sizeof(LinePass));
    if (!rc) rc = balloc(b, (void **)&b->d_fp, fp.size() * sizeof(FusedPass));
    if (!rc) rc = balloc(b, (void **)&b->d_zf, (size_t)count * sizeof(ZFwdArgs));
    if (!rc) rc = balloc(b, (void **)&b->d_zi, (size_t)5 * count * sizeof(ZInvArgs));
    if (!rc) {
        hipError_t e = hipMemcpy(b->d_lpf, lf.data(), lf.size() * sizeof(LinePass), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_lpi, li.data(), li.size() * sizeof(LinePass), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_fp, fp.data(), fp.size() * sizeof(FusedPass), hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = fail(MM_EHIP, "batch tables: %s", hipGetErrorString(e));
    }
    if (!rc) {
        const int tm = tune_mode(o.autotune);
        rc = precision == MM_F32 ? batch_autotune<float>(b, tm) : batch_autotune<double>(b, tm);
    }
    if (rc) {
        std::string keep = g_last;
        batch_free(b);
        delete b;
        g_last = keep;
        return rc;
    }
    *out = b;
    return MM_OK;
}

int mm_batch_h_eff(mm_batch *b, void *const *m_ptrs, const double *Ms, double A, void *const *h_ptrs, unsigned terms) {
    if (!b) return fail(MM_EINVAL, "batch is NULL");
    if (!m_ptrs || !Ms || !h_ptrs) return fail(MM_EINVAL, "m_ptrs, Ms and h_ptrs must be non-NULL");
    if (terms == 0 || (terms & ~(MM_DEMAG | MM_EXCHANGE))) return fail(MM_EINVAL, "bad terms");
    for (int g = 0; g < b->count; ++g) {
        if (!m_ptrs[g] || !h_ptrs[g] || m_ptrs[g] == h_ptrs[g]) return fail(MM_EINVAL, "geometry %d: bad m/h pointer", g);
        if (!(Ms[g] >= 0.0) || !std::isfinite(Ms[g])) return fail(MM_EINVAL, "geometry %d: Ms must be finite and >= 0", g);
    }
    if (!std::isfinite(A) || A < 0) return fail(MM_EINVAL, "A must be finite and >= 0");
    int rc = batch_args(b, m_ptrs, Ms, A, 0.0, 1.0, 1.0, h_ptrs, terms, 1);
    if (rc) return rc;
    b->akey.clear();   // the stage arguments now differ from any captured graph's
    return b->prec == MM_F32 ? batch_heff<float>(b, terms) : batch_heff<double>(b, terms);
}

int mm_batch_llg_step(mm_batch *b, void *const *m_ptrs, const double *Ms, double A, double alpha, double gamma,
                      double dt, int n_steps, unsigned flags) {
    if (!b) return fail(MM_EINVAL, "batch is NULL");
    if (!m_ptrs || !Ms) return fail(MM_EINVAL, "m_ptrs and Ms must be non-NULL");
    if (n_steps < 0) return fail(MM_EINVAL, "n_steps must be >= 0");
    if (flags & ~(MM_NO_RENORM | MM_NO_GRAPH)) return fail(MM_EINVAL, "unknown flags");
    for (int g = 0; g < b->count; ++g) {
        if (!m_ptrs[g]) return fail(MM_EINVAL, "geometry %d: m is NULL", g);
        if (!(Ms[g] >= 0.0) || !std::isfinite(Ms[g])) return fail(MM_EINVAL, "geometry %d: Ms must be finite and >= 0", g);
    }
    if (!std::isfinite(A) || A < 0) return fail(MM_EINVAL, "A must be finite and >= 0");
    int rc = check_llg(alpha, gamma, dt, nullptr);
    if (rc) return rc;
    if (n_steps == 0) return MM_OK;
    const int renorm = (flags & MM_NO_RENORM) ? 0 : 1;
    std::vector<unsigned char> key = batch_key(b, m_ptrs, Ms, A, alpha, gamma, dt, nullptr, 3u, renorm);
    if (key != b->akey) {
        if ((rc = batch_args(b, m_ptrs, Ms, A, alpha, gamma, dt, nullptr, 3u, renorm))) return rc;
        b->akey = key;
    }
    if (flags & MM_NO_GRAPH) {
        for (int k = 0; k < n_steps; ++k) {
            rc = b->prec == MM_F32 ? batch_step<float>(b) : batch_step<double>(b);
            if (rc) return rc;
        }
        return MM_OK;
    }
    if (!b->gexec || key != b->gkey) {
        if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
        hipGraph_t graph = nullptr;
        if (!b->cap) HIPCK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        hipStream_t user = b->stream;
        b->stream = b->cap;
        hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) { b->stream = user; return fail(MM_EHIP, "begin capture: %s", hipGetErrorString(e)); }
        rc = b->prec == MM_F32 ? batch_step<float>(b) : batch_step<double>(b);
        e = hipStreamEndCapture(b->cap, &graph);
        b->stream = user;
        if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
        if (e != hipSuccess) return fail(MM_EHIP, "batch graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) { b->gexec = nullptr; return fail(MM_EHIP, "batch graph instantiate: %s", hipGetErrorString(e)); }
        b->gkey = key;
    }
    for (int k = 0; k < n_steps; ++k) HIPCK(hipGraphLaunch(b->gexec, b->stream));
    return MM_OK;
}

int mm_batch_tensor_set(mm_batch *b, int geometry, const double *host_octant) {
    if (!b) return fail(MM_EINVAL, "batch is NULL");
    if (geometry < 0 || geometry >= b->count) return fail(MM_EINVAL, "geometry %d out of range [0, %d)", geometry, b->count);
    HIPCK(hipStreamSynchronize(b->stream));
    // the plan's spectrum buffer stays where the batch's descriptors point
    return mm_demag_tensor_set(b->plans[geometry], host_octant);
}

int mm_batch_info(const mm_batch *b, int64_t *total_cells, size_t *device_bytes) {
    if (!b) return fail(MM_EINVAL, "batch is NULL");
    int64_t n = 0;
    size_t by = b->bytes;
    for (const mm_plan *p : b->plans) { n += p->n[0] * p->n[1] * p->n[2]; by += p->bytes; }
    if (total_cells) *total_cells = n;
    if (device_bytes) *device_bytes = by;
    return MM_OK;
}

int mm_batch_schedule(const mm_batch *b, char *buf, size_t len) {
    if (!b) return fail(MM_EINVAL, "batch is NULL");
    std::string t = "{\"groups\": [";
    bool first = true;
    auto add = [&](const char *pass, const std::vector<BGroup> &gs) {
        for (const BGroup &g : gs) {
            char s[256];
            snprintf(s, sizeof s, "%s{\"pass\": \"%s\", \"L\": %d, \"specialised\": %d, \"variant\": %d, \"W\": %d, "
                     "\"geometries\": %zu, \"tiles\": %d}", first ? "" : ", ", pass, g.L ? g.L : 0, g.L ? 1 : 0, g.var, g.W,
                     g.geo.size(), g.tiles);
            t += s;
            first = false;
        }
    };
    add("x_fwd", b->gxf);
    add("y_fused", b->gy);
    add("x_inv", b->gxi);
    add("z", b->gz);
    t += "]}";
    return put_text(t, buf, len);
}

int mm_batch_destroy(mm_batch *b) {
    if (!b) return fail(MM_EINVAL, "batch is NULL");
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    delete b;
    return MM_OK;
}

}  // extern "C"
