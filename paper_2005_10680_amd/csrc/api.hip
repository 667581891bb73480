// C ABI of the library (include/spamm.h): argument validation, workspace
// carving and the purification driver.  Kernels live in the other .hip files.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <string>
#include <vector>

#include "../../include/spamm.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace spamm;

namespace spamm {
// small-system single-workgroup passes (on by default)
static std::atomic<bool> g_small_path{true};
bool small_path_enabled() { return g_small_path.load(std::memory_order_relaxed); }
void set_small_path(bool on) { g_small_path.store(on, std::memory_order_relaxed); }
}  // namespace spamm

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(SPAMM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int ceil_log2(int x) {
    int L = 0;
    while ((1 << L) < x) ++L;
    return L;
}

int num_cus() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) cached = p.multiProcessorCount;
        else cached = 256;
    }
    return cached;
}

// Streams kept for the purifications: one per host thread, device and use
// (0: the stream a graph is captured on, 1: the side stream of the
// split-BF16 copies), created on first use and kept until the process ends
// (creating and destroying one per call costs about as much as a small
// system's whole loop).  Calls on one thread run one after another, so they
// never share one at the same time.  Default priority.
static hipError_t kept_stream(int use, hipStream_t* out) {
    constexpr int kMaxDev = 64;
    thread_local hipStream_t streams[2][kMaxDev] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
    if (!streams[use][dev]) {
        e = hipStreamCreateWithFlags(&streams[use][dev], hipStreamNonBlocking);
        if (e != hipSuccess) return e;
    }
    *out = streams[use][dev];
    return hipSuccess;
}

hipError_t capture_stream(hipStream_t* out) { return kept_stream(0, out); }

// Graph, executable graph and event of one device-driven loop; a capture
// left open by an early return is ended first, so the kept stream stays
// usable.
struct GraphGuard {
    hipStream_t cs = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipEvent_t e = nullptr;
    ~GraphGuard() {
        if (cs) {
            hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(cs, &st) == hipSuccess && st != hipStreamCaptureStatusNone) {
                hipGraph_t open = nullptr;
                if (hipStreamEndCapture(cs, &open) == hipSuccess && open) (void)hipGraphDestroy(open);
            }
        }
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
        if (e) (void)hipEventDestroy(e);
    }
};

// Pair lists use 32-bit offsets: a capacity derived from the workspace is
// capped below 2^31, so that a longer list reports SPAMM_ECAPACITY.
int64_t clamp_pairs(int64_t max_pairs) {
    const int64_t lim = ((int64_t)1 << 31) - 1;
    return max_pairs < lim ? max_pairs : lim;
}

int check_bsm(const spamm_bsm* X, const char* name, bool need_norms) {
    if (!X) return fail(SPAMM_EINVAL, "%s is NULL", name);
    if (X->n <= 0) return fail(SPAMM_EINVAL, "%s: n must be positive", name);
    if (X->b != 32 && X->b != 64 && X->b != 128) return fail(SPAMM_EINVAL, "%s: leaf size must be 32, 64 or 128", name);
    if ((int64_t)X->nb != (X->n + X->b - 1) / X->b) return fail(SPAMM_EINVAL, "%s: nb != ceil(n/b)", name);
    if (X->nb > 2048) return fail(SPAMM_EINVAL, "%s: nb > 2048 is not supported", name);
    if (X->cap < 0) return fail(SPAMM_EINVAL, "%s: negative capacity", name);
    if (!X->nslot || !X->brow || !X->bcol || !X->map || !X->val)
        return fail(SPAMM_EINVAL, "%s: NULL array", name);
    if (need_norms && (!X->norm || !X->sq || !X->sqlo)) return fail(SPAMM_EINVAL, "%s: NULL norm arrays", name);
    return SPAMM_OK;
}

MatView view(const spamm_bsm* X) {
    MatView v;
    v.n = X->n;
    v.b = X->b;
    v.nb = X->nb;
    v.cap = X->cap;
    v.nslot = X->nslot;
    v.brow = X->brow;
    v.bcol = X->bcol;
    v.map = X->map;
    v.val = X->val;
    v.norm = X->norm;
    v.sq = X->sq;
    v.sqlo = X->sqlo;
    return v;
}

struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <class T>
    T* take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

// ---------------------------------------------------------------------------
// sweep workspace
// ---------------------------------------------------------------------------
struct SweepWs {
    int nb, L, l0, T;
    int64_t ncap;
    uint8_t *tA, *tB;
    int32_t *flag, *idx, *lflag, *lpos, *pstart;
    uint32_t* keys[2];
    double* vals[2];
    int64_t* cnt;  // [4]
    int32_t* ovf;
    void* scan_tmp;
    // leaf-level bounds (B_flat, B_sum)
    int nw;
    uint32_t *bitsA, *bitsB;
    void* part;     // the leaf-level bounds' partial sums and exact accumulators
    double* bleaf;  // [N]
    int64_t* one;
};

void carve_sweep(Carver& c, int nb, int N, SweepWs& w) {
    w.nb = nb;
    w.L = ceil_log2(nb);
    w.l0 = cse_level0(nb);
    w.T = 1 << (w.L - w.l0);
    w.ncap = (int64_t)w.T * w.T * w.T;
    w.tA = c.take<uint8_t>((size_t)w.T * w.T);
    w.tB = c.take<uint8_t>((size_t)w.T * w.T);
    w.flag = c.take<int32_t>(w.ncap);
    w.idx = c.take<int32_t>(w.ncap);
    w.lflag = c.take<int32_t>(w.ncap);
    w.lpos = c.take<int32_t>(w.ncap);
    w.pstart = c.take<int32_t>(w.ncap + 1);
    w.keys[0] = c.take<uint32_t>(w.ncap);
    w.keys[1] = c.take<uint32_t>(w.ncap);
    w.vals[0] = c.take<double>((size_t)w.ncap * N);
    w.vals[1] = c.take<double>((size_t)w.ncap * N);
    w.cnt = c.take<int64_t>(4);
    w.ovf = c.take<int32_t>(4);
    w.scan_tmp = c.take<char>(scan_temp_bytes(w.ncap));
    w.nw = (nb + 31) / 32;
    w.bitsA = c.take<uint32_t>((size_t)nb * w.nw);
    w.bitsB = c.take<uint32_t>((size_t)nb * w.nw);
    w.part = c.take<char>(bound_leaf_scratch_bytes(nb, N));
    w.bleaf = c.take<double>(N);
    w.one = c.take<int64_t>(1);
}

// Occupancy of a matrix X with a symmetric block pattern, for the products
// X X^T of the purification (A = X, B given transposed as X): the row
// bitmaps (nw words per block row) and the level-l0 tiles of X serve as both
// operands' (the tiles of X^T are the transposed tiles of X, equal for a
// symmetric pattern), so one pass builds what the sweep and the kept pairs
// would otherwise build four times.
struct SymOcc {
    const uint32_t* bits;
    const uint8_t* tiles;
    bool cubes;  // the sweep's cube list of X X^T is in sw->keys[0] / sw->cnt[0]
};

// With sw given and a small X, one workgroup builds the occupancy and the
// sweep's cube list (the sweeps of the step then start at the cube pass;
// for nb <= kSmallNb no level pass runs below the top levels, so the list
// stays intact across the step's sweeps).
SymOcc build_sym_occ(const MatView& X, uint32_t* bits, int nw, uint8_t* tiles, int T, int l0, const int32_t* done,
                     hipStream_t s, SweepWs* sw = nullptr) {
    if (X.nb <= kSmallNb && T <= kSmallTiles && small_path_enabled()) {
        launch_occ_small(X, bits, nw, tiles, T, l0, sw ? sw->keys[0] : nullptr, sw ? &sw->cnt[0] : nullptr, done, s);
        return SymOcc{bits, tiles, sw != nullptr};
    }
    fill_u32(bits, (int64_t)X.nb * nw, 0u, s);
    fill_u8(tiles, (int64_t)T * T, 0, s);
    launch_occupancy(X, kOccA, bits, nw, tiles, T, l0, done, s);
    return SymOcc{bits, tiles, false};
}

// The leaf-level bounds B_flat (kind 1) or B_sum (kind 2) for every
// candidate (mode 1: the tier mode, as in run_sweep), then the selection rule.
// occ: precomputed occupancy of A = B (symmetric pattern), or null.
void run_sweep_leaf(const MatView& A, const MatView& B, int btrans, const double* tau, int N,
                    const double* budget_dev, double budget_host, int kind, int mode, const double* tau0_dev,
                    double c_low, double* bound_out, int32_t* idx_out, double* tau_out, SweepWs& w,
                    const int32_t* done, hipStream_t s, const SymOcc* occ = nullptr) {
    const int nb = A.nb;
    const uint32_t* bA = w.bitsA;
    const uint32_t* bB = w.bitsB;
    if (occ) {
        bA = bB = occ->bits;
    } else {
        fill_u32(w.bitsA, (int64_t)nb * w.nw, 0u, s);
        fill_u32(w.bitsB, (int64_t)nb * w.nw, 0u, s);
        launch_occupancy(A, kOccA, w.bitsA, w.nw, nullptr, 0, 0, done, s);
        launch_occupancy(B, btrans ? kOccBt : kOccB, w.bitsB, w.nw, nullptr, 0, 0, done, s);
    }
    launch_bound_leaf(nb, w.nw, bA, bB, A.map, A.norm, B.map, B.norm, btrans, tau, N, kind == 1 ? 1 : 0,
                      mode, tau0_dev, c_low, w.part, w.bleaf, done, s);
    fill_i64(w.one, 1, 1, s);
    launch_select(w.bleaf, w.one, tau, N, budget_dev, budget_host, bound_out, idx_out, tau_out, done, s);
}

void run_sweep(const MatView& A, const MatView& B, int btrans, const double* tau, int N, const double* budget_dev,
               double budget_host, int mode, const double* tau0, double c_low, double* bound_out, int32_t* idx_out,
               double* tau_out, SweepWs& w, const int32_t* done, hipStream_t s, const SymOcc* occ = nullptr) {
    const int T = w.T;
    if (occ && occ->cubes) {
        // cube list already built with the occupancy
    } else if (occ) {
        launch_cube_flags(T, occ->tiles, occ->tiles, w.flag, done, s);
    } else {
        fill_u8(w.tA, (int64_t)T * T, 0, s);
        fill_u8(w.tB, (int64_t)T * T, 0, s);
        launch_occupancy(A, kOccA, nullptr, 0, w.tA, T, w.l0, done, s);
        launch_occupancy(B, btrans ? kOccBt : kOccB, nullptr, 0, w.tB, T, w.l0, done, s);
        launch_cube_flags(T, w.tA, w.tB, w.flag, done, s);
    }
    if (!(occ && occ->cubes)) {
        scan_i32(w.flag, w.idx, w.ncap, nullptr, &w.cnt[0], w.scan_tmp, s);
        launch_cube_list(T, w.flag, w.idx, w.keys[0], &w.cnt[0], w.ncap, w.ovf, done, s);
    }
    launch_cube_eval(mode, w.l0, A.nb, w.keys[0], &w.cnt[0], w.ncap, A.map, A.norm, B.map, B.norm, btrans, tau, N,
                     tau0, c_low, w.vals[0], done, s);
    // levels whose children may number more than kTopNodes (8^4) run as
    // separate device-wide passes; the rest, and the selection, in one
    // workgroup
    const int top = std::max(w.l0 + 1, w.L - 3);
    int cur = 0;
    for (int lev = w.l0 + 1; lev < top; ++lev) {
        int64_t* nc = &w.cnt[cur];
        int64_t* np = &w.cnt[1 - cur];
        launch_level_flags(w.keys[cur], nc, w.ncap, w.lflag, done, s);
        scan_i32(w.lflag, w.lpos, w.ncap, nc, np, w.scan_tmp, s);
        launch_level_build(w.keys[cur], nc, w.ncap, w.lflag, w.lpos, np, w.keys[1 - cur], w.pstart, done, s);
        launch_level_eval(w.keys[cur], w.vals[cur], w.pstart, np, w.ncap, N, w.vals[1 - cur], done, s);
        cur = 1 - cur;
    }
    launch_levels_top(w.keys[cur], &w.cnt[cur], w.vals[cur], w.vals[1 - cur], std::max(0, w.L - top + 1), N, tau,
                      budget_dev, budget_host, bound_out, idx_out, tau_out, done, s);
}

// ---------------------------------------------------------------------------
// multiply workspace
// ---------------------------------------------------------------------------
struct MulWs {
    int nb, P, nw;
    int64_t PP, cap_out, cap_pairs;
    uint32_t *bitsA, *bitsB;
    int32_t *cnt, *cflag, *off, *oidx, *oi, *oj, *optr, *hflag, *hslot, *cnt_low, *olow;
    int2* pairs;
    int64_t* sc;  // [8]: npairs, nout, nslot_total
    int32_t* counters;
    int32_t* cuts;  // [9] per-XCD output ranges, written by the small-system pair pass
    int32_t* ovf;
    void* scan_tmp;
    bool counters_clear = false;  // the last pair pass cleared the work counters and wrote cuts
};

void carve_mul(Carver& c, int nb, int64_t max_pairs, MulWs& w) {
    w.nb = nb;
    w.P = 1 << ceil_log2(nb);
    w.nw = (nb + 31) / 32;
    w.PP = (int64_t)w.P * w.P;
    w.cap_out = (int64_t)nb * nb;
    w.cap_pairs = max_pairs;
    w.bitsA = c.take<uint32_t>((size_t)nb * w.nw);
    w.bitsB = c.take<uint32_t>((size_t)nb * w.nw);
    w.cnt = c.take<int32_t>(w.PP);
    w.cflag = c.take<int32_t>(w.PP);
    w.off = c.take<int32_t>(w.PP);
    w.oidx = c.take<int32_t>(w.PP);
    w.hflag = c.take<int32_t>(w.PP);
    w.hslot = c.take<int32_t>(w.PP);
    w.oi = c.take<int32_t>(w.cap_out);
    w.oj = c.take<int32_t>(w.cap_out);
    w.optr = c.take<int32_t>(w.cap_out + 1);
    w.cnt_low = c.take<int32_t>(w.PP);
    w.olow = c.take<int32_t>(w.cap_out);
    w.pairs = c.take<int2>(w.cap_pairs > 0 ? w.cap_pairs : 1);
    w.sc = c.take<int64_t>(8);
    w.counters = c.take<int32_t>(16);
    w.cuts = c.take<int32_t>(16);
    w.ovf = c.take<int32_t>(4);
    w.scan_tmp = c.take<char>(scan_temp_bytes(w.PP));
}

// Kept pairs of SpAMM(A, B, *tau) and the output pattern written into C
// (map, brow, bcol, nslot); with X given, the pattern of 2X - C (branch 1).
void run_pairs(const MatView& A, const MatView& B, int btrans, int sym, const double* tau_dev, const double* sigma_dev,
               const MatView& C, uint8_t* fromc, MulWs& w, const int32_t* mapX, const int32_t* branch_dev,
               const int32_t* done, hipStream_t s, const SymOcc* occ = nullptr, double norm_min = 0.0) {
    const int nb = A.nb;
    const uint32_t* bA = w.bitsA;
    const uint32_t* bB = w.bitsB;
    if (occ) {
        bA = bB = occ->bits;
    } else {
        fill_u32(w.bitsA, (int64_t)nb * w.nw, 0u, s);
        fill_u32(w.bitsB, (int64_t)nb * w.nw, 0u, s);
        launch_occupancy(A, kOccA, w.bitsA, w.nw, nullptr, 0, 0, done, s);
        launch_occupancy(B, btrans ? kOccBt : kOccB, w.bitsB, w.nw, nullptr, 0, 0, done, s);
    }
    if (nb <= kSmallNb && small_path_enabled()) {
        launch_pairs_small(nb, w.P, w.nw, bA, bB, A.map, A.norm, B.map, B.norm, btrans, sym, tau_dev, sigma_dev,
                           norm_min, w.cap_pairs, w.cap_out, w.oi, w.oj, w.optr, w.pairs, sigma_dev ? w.olow : nullptr,
                           w.sc, C.cap, C.map, C.brow, C.bcol, C.nslot, fromc, mapX, branch_dev, w.counters, w.cuts,
                           w.ovf, done, s);
        w.counters_clear = true;
        return;
    }
    w.counters_clear = false;
    launch_kept_count(nb, w.P, w.nw, bA, bB, A.map, A.norm, B.map, B.norm, btrans, sym, tau_dev, sigma_dev,
                      norm_min, w.cnt, w.cflag, sigma_dev ? w.cnt_low : nullptr, done, s);
    scan_i32(w.cnt, w.off, w.PP, nullptr, &w.sc[0], w.scan_tmp, s);
    scan_i32(w.cflag, w.oidx, w.PP, nullptr, &w.sc[1], w.scan_tmp, s);
    if (sigma_dev) scan_i32(w.cnt_low, w.hslot, w.PP, nullptr, &w.sc[3], w.scan_tmp, s);  // total low pairs
    else fill_i64(&w.sc[3], 1, 0, s);
    launch_kept_fill(nb, w.P, w.nw, bA, bB, A.map, A.norm, B.map, B.norm, btrans, tau_dev, sigma_dev, norm_min, w.cnt,
                     w.off, w.oidx, &w.sc[0], &w.sc[1], w.cap_pairs, w.cap_out, w.oi, w.oj, w.optr, w.pairs,
                     sigma_dev ? w.olow : nullptr, w.ovf, done, s);
    launch_hat_flags(nb, w.P, w.cnt, sym, mapX, branch_dev, w.hflag, done, s);
    scan_i32(w.hflag, w.hslot, w.PP, nullptr, &w.sc[2], w.scan_tmp, s);
    launch_hat_assign(nb, w.P, w.cnt, sym, w.hflag, w.hslot, &w.sc[2], C.cap, C.map, C.brow, C.bcol, C.nslot, fromc,
                      w.ovf, done, s);
}

// Leaf products of the kept pairs into C's slots (combined with X when given);
// with no.sq also the norms of the written blocks (the product's work
// counters, reset before the product, hold the recheck count at [8]).
// With out32 also the FP32 copies of the written blocks (FP32 tier).
// Returns -1 only for norms or copies requested without the transposed-B
// layout (copies: without the FP32 tier).
int run_gemm(const MatView& A, const MatView& B, int btrans, int sym, const MatView& C, const uint8_t* fromc,
              MulWs& w, const int32_t* mapX, const double* valX, const int32_t* branch_dev, const int32_t* done,
              hipStream_t s, const float* valA32 = nullptr, const float* valB32 = nullptr,
              hipEvent_t ev_start = nullptr, hipEvent_t ev_end = nullptr, const uint16_t* valA16 = nullptr,
              const uint16_t* valB16 = nullptr, const int32_t* expA = nullptr, const int32_t* expB = nullptr,
              NormOut no = NormOut(), float* out32 = nullptr) {
    const int nb = A.nb;
    GemmArgs g;
    g.b = A.b;
    g.nb = nb;
    g.oi = w.oi;
    g.oj = w.oj;
    g.optr = w.optr;
    g.pairs = w.pairs;
    g.nout = &w.sc[1];
    g.npairs = &w.sc[0];
    g.valA = A.val;
    g.valB = B.val;
    g.btrans = btrans;
    g.sym = sym;
    g.map_out = C.map;
    g.val_out = C.val;
    g.mapX = mapX;
    g.valX = valX;
    g.branch = branch_dev;
    g.counters = w.counters;
    g.ovf = w.ovf;
    g.done = done;
    g.valA32 = valA32;
    g.valB32 = valB32;
    g.valA16 = valA16;
    g.valB16 = valB16;
    g.expA = expA;
    g.expB = expB;
    g.olow = (valA32 || valA16) ? w.olow : nullptr;
    if (no.sq) {
        // block norms in the product's epilogue (the ring kernels of the
        // transposed-B layout only)
        if (!btrans) return -1;
        g.sq_out = no.sq;
        g.sqlo_out = no.sqlo;
        g.nrm_out = no.nrm;
        g.recheck = no.recheck;
        g.nrecheck = no.nrecheck;
    }
    if (out32) {
        // FP32 copies of the outputs in the epilogue (the FP32-tier ring kernels)
        if (!btrans || !valA32) return -1;
        g.out32 = out32;
    }
    if (w.counters_clear) g.cuts = w.cuts;
    launch_gemm_f64(g, num_cus(), s, ev_start, ev_end, w.counters_clear);
    w.counters_clear = false;
    if (mapX)
        launch_rest(A.b, C.nslot, C.cap, C.brow, C.bcol, fromc, nb, mapX, valX, C.val, branch_dev, done, s, no, out32);
    return 0;
}

// ---------------------------------------------------------------------------
// host copies of the decision rules of the driver (same arithmetic as the
// algorithm's statement; double precision, one rounding per operation)
// ---------------------------------------------------------------------------
double step_delta(const sp2_params* p, double gap) {
    return sp2_step_delta(p->eps, p->n_max, p->delta_const, gap);
}
int choose_branch(double t1, double t2, int64_t n_occ) { return sp2_choose_branch(t1, t2, n_occ); }
double map_gap(double x, int br) { return sp2_map_gap(x, br); }
bool should_stop(const std::vector<double>& eh, double e_tol) {
    double e[3];
    const int n = (int)std::min<size_t>(eh.size(), 3);
    for (int q = 0; q < n; ++q) e[q] = eh[eh.size() - 1 - q];
    return sp2_should_stop(e, n, e_tol);
}

// c_t of the FP32 tier: inputs rounded to FP32 (u = 2^-24 each), products
// of length b accumulated by the FP32 MFMA with an assumed unit roundoff of
// 2u (no better than round-to-nearest is assumed), so
// |fl(AB) - AB| <= (2u + u^2 + gamma_b(2u)(1+u)^2) |A||B| entrywise and
// ||fl(AB) - AB||_F <= c ||A||_F ||B||_F.  Rounded up by 2^-40.
double tier_constant(int precision, int b) {
    const double m = (double)b;
    if (precision == 1) {
        // operands rounded to FP32, b products accumulated in FP32 (unit
        // roundoff 2^-23 assumed); 2^-31 covers entries and partial results
        // below the FP32 normal range, with both block norms >= kFp32TierNormMin
        const double u = 0x1p-24, ue = 2.0 * u;
        const double gam = m * ue / (1.0 - m * ue);
        return (2.0 * u + u * u + gam * (1.0 + u) * (1.0 + u) + 0x1p-31) * (1.0 + 0x1p-40);
    }
    if (precision == 2) {
        // split BF16: x = hi + lo + e after a power-of-two block scaling,
        // |lo| <= u (1+u) |x|, |e| <= u^2 (1+u) |x| (u = 2^-8); dropped terms
        // lo lo', e (hi' + lo'), (hi + lo) e', e e'; the three products exact
        // in FP32, 3b terms accumulated in FP32 (unit roundoff 2^-23 assumed);
        // 2^-100 covers entries below the BF16 normal range
        const double u = 0x1p-8, ue = 2.0 * 0x1p-24;
        const double kappa = u * u * (pow(1.0 + u, 2.0) + 2.0 * pow(1.0 + u, 3.0) + u * u * pow(1.0 + u, 2.0));
        const double gam = 3.0 * m * ue / (1.0 - 3.0 * m * ue);
        return (kappa + gam * (1.0 + 2.0 * u) * pow(1.0 + u, 2.0) + 0x1p-100) * (1.0 + 0x1p-40);
    }
    return 0.0;
}

double trunc_quantum(double delta) { return sp2_trunc_quantum(delta); }

__global__ void k_trunc_report(const int64_t* stats, const double* delta_dev, double delta_host, double scale,
                               double* out) {
    const double delta = (delta_dev ? *delta_dev : delta_host) * scale;
    const double T = delta * delta;
    double Q = 0.0;
    if (T > 0.0 && isfinite(T)) {
        int e;
        frexp(T, &e);
        int eq = e - 1 - 40;
        if (eq < -1000) eq = -1000;
        Q = ldexp(1.0, eq);
    }
    out[0] = (double)stats[0];
    out[1] = (double)stats[1] * Q;
}

void carve_mat(Carver& c, int64_t n, int b, int64_t cap, spamm_bsm& m) {
    m.n = n;
    m.b = b;
    m.nb = (int32_t)((n + b - 1) / b);
    m.cap = cap;
    m.nslot = c.take<int32_t>(1);
    m.brow = c.take<int32_t>(cap);
    m.bcol = c.take<int32_t>(cap);
    m.map = c.take<int32_t>((size_t)m.nb * m.nb);
    m.val = c.take<double>((size_t)cap * b * b);
    m.norm = c.take<double>(cap);
    m.sq = c.take<double>(cap);
    m.sqlo = c.take<double>(cap);
}

// dst = src (pattern, values, norms); both with capacity cap
int copy_mat(const spamm_bsm& dst, const spamm_bsm& src, int64_t cap, hipStream_t s) {
    launch_copy_live(view(&src), view(&dst), cap, s);
    HIP_TRY(hipGetLastError());
    return SPAMM_OK;
}

struct Sp2Ws {
    spamm_bsm X[2];
    std::vector<spamm_bsm> tape;
    SweepWs sw;
    MulWs mw;
    uint8_t* fromc;
    void* trunc_tmp;
    int64_t* tstats;  // [4]
    double* trace_tmp;
    double* trace_out;  // [4]
    double* rowtmp;     // [2n]
    double* lam;        // [2]
    int32_t* dflag;
    int32_t* dpos;
    int64_t* dcount;
    double* bound;  // [N]
    double* bound2; // [N] sweep over the low-precision limit
    float* x32;     // FP32 copy of the current iterate (FP32 tier), or its split-BF16 parts
    int32_t* xexp;  // per-slot exponents of the split-BF16 parts
    int32_t* recheck;  // [cap] slots whose norm the product kernels left to the norms kernel
    float* x32n;       // FP32 tier, one system: the copy of the next iterate, written by the product
    Sp2Ctl* ctl;
    sp2_iter_log* dlog;  // [kMaxLog] records written by the device control (graph mode)
};

// product groups of a batch: (leaf size, tier) pairs; leaf 32, 64, 128 in
// FP64, leaf 32 and 64 in the two tiers
constexpr int kBatchGroups = 7;
constexpr int kMaxLog = 10002;  // n_max <= 10000, plus the stop record

// the control step of the device-driven loop, run by the traces launch
TraceTail control_tail(const Sp2Ws& w) {
    TraceTail t;
    t.ctl = w.ctl;
    t.msc = w.mw.sc;
    t.ts = w.tstats;
    t.ovf_mul = w.mw.ovf;
    t.ovf_sweep = w.sw.ovf;
    t.logs = w.dlog;
    t.max_records = kMaxLog;
    return t;
}

// x1_outside: the second iterate buffer X[1] is not carved (the batched
// loop uses the caller's output matrix for it)
void carve_sp2(Carver& c, int nb, int b, int N, int64_t cap, int64_t max_pairs, int tape_steps, Sp2Ws& w,
               int precision = 0, bool x1_outside = false) {
    const int64_t n = (int64_t)nb * b;
    carve_mat(c, n, b, cap, w.X[0]);
    if (!x1_outside) carve_mat(c, n, b, cap, w.X[1]);
    w.tape.resize(tape_steps > 0 ? tape_steps + 1 : 0);
    for (auto& t : w.tape) carve_mat(c, n, b, cap, t);
    carve_sweep(c, nb, N, w.sw);
    carve_mul(c, nb, max_pairs, w.mw);
    w.fromc = c.take<uint8_t>(cap);
    w.trunc_tmp = c.take<char>(trunc_temp_bytes(cap));
    w.tstats = c.take<int64_t>(4);
    w.trace_tmp = c.take<double>(traces_temp_bytes() / sizeof(double));
    w.trace_out = c.take<double>(4);
    w.rowtmp = c.take<double>(2 * (size_t)n);
    w.lam = c.take<double>(2);
    w.dflag = c.take<int32_t>(nb);
    w.dpos = c.take<int32_t>(nb);
    w.dcount = c.take<int64_t>(2);
    w.bound = c.take<double>(N);
    w.bound2 = c.take<double>(N);
    w.ctl = c.take<Sp2Ctl>(1);
    w.dlog = c.take<sp2_iter_log>(kMaxLog);
    w.x32 = precision ? c.take<float>((size_t)cap * b * b) : nullptr;
    w.xexp = precision == 2 ? c.take<int32_t>(cap) : nullptr;
    w.recheck = c.take<int32_t>(cap);
    w.x32n = (precision == 1 && !x1_outside) ? c.take<float>((size_t)cap * b * b) : nullptr;
}

// argument checks shared by the single and the batched purification
int check_sp2(const spamm_bsm* F, const sp2_params* p, const spamm_bsm* D) {
    int rc = check_bsm(F, "F", false);
    if (!rc) rc = check_bsm(D, "D", true);
    if (rc) return rc;
    if (!p) return fail(SPAMM_EINVAL, "NULL parameters");
    if (D->nb != F->nb || D->b != F->b || D->n != F->n) return fail(SPAMM_EINVAL, "D must match F");
    if (p->n_max < 1 || p->n_max > 10000) return fail(SPAMM_EINVAL, "n_max out of range");
    if (p->variant < 0 || p->variant > 2) return fail(SPAMM_EINVAL, "variant must be 0, 1 or 2");
    if (p->N < 1 || p->N > 1024 || !p->tau) return fail(SPAMM_EINVAL, "bad candidate list");
    if (p->n_occ < 0 || p->n_occ > F->n) return fail(SPAMM_EINVAL, "n_occ out of range");
    const bool have_gap = !isnan(p->homo) && !isnan(p->lumo);
    if (!have_gap && isnan(p->delta_const)) return fail(SPAMM_EINVAL, "need homo/lumo or delta_const");
    if (have_gap && !(p->homo < p->lumo)) return fail(SPAMM_EINVAL, "need homo < lumo");
    if (!(p->eps > 0.0)) return fail(SPAMM_EINVAL, "eps must be > 0");
    if (p->precision < 0 || p->precision > 2)
        return fail(SPAMM_EINVAL, "precision must be 0 (FP64), 1 (FP32 tier) or 2 (split-BF16 tier)");
    if (p->graph_steps < 0) return fail(SPAMM_EINVAL, "graph_steps must be >= 0");
    if (p->graph_steps > 0 && p->keep_tape) return fail(SPAMM_EINVAL, "graph mode needs keep_tape = 0");
    if (p->keep_tape < 0 || p->keep_tape > p->n_max) return fail(SPAMM_EINVAL, "keep_tape must be in 0..n_max");
    if (p->bound_kind < 0 || p->bound_kind > 2) return fail(SPAMM_EINVAL, "bound_kind must be 0, 1 or 2");
    if (p->bound_kind != 0 && F->nb > kBoundMaxNb)
        return fail(SPAMM_ENOTSUP, "the leaf-level bounds support nb <= %d", kBoundMaxNb);
    if (p->precision != 0 && F->b > 64) return fail(SPAMM_ENOTSUP, "the precision tiers support leaf 32 and 64");
    if (p->precision != 0 && !(p->tier_split > 0.0 && p->tier_split < 1.0))
        return fail(SPAMM_EINVAL, "tier_split must be in (0, 1)");
    return SPAMM_OK;
}

// ---------------------------------------------------------------------------
// adjoint workspace: one reverse step (pair list on the pattern of X)
// ---------------------------------------------------------------------------
struct AdjWs {
    int nb, nw;
    int64_t cap, cap_pairs;
    uint32_t *bitsX, *bitsG;
    int32_t *flag, *pos, *oi, *oj, *cnt, *optr;
    int2* pairs;
    int64_t* sc;        // [0] outputs, [1] pairs
    int32_t* counters;  // [16]
    int32_t* ovf;       // [4]
    int32_t* branch;    // [1]
    void* scan_tmp;
};

void carve_adj(Carver& c, int nb, int64_t cap, int64_t max_pairs, AdjWs& w) {
    w.nb = nb;
    w.nw = (nb + 31) / 32;
    w.cap = cap;
    w.cap_pairs = max_pairs;
    w.bitsX = c.take<uint32_t>((size_t)nb * w.nw);
    w.bitsG = c.take<uint32_t>((size_t)nb * w.nw);
    w.flag = c.take<int32_t>(cap);
    w.pos = c.take<int32_t>(cap);
    w.oi = c.take<int32_t>(cap);
    w.oj = c.take<int32_t>(cap);
    w.cnt = c.take<int32_t>(cap);
    w.optr = c.take<int32_t>(cap + 1);
    w.sc = c.take<int64_t>(4);
    w.counters = c.take<int32_t>(16);
    w.ovf = c.take<int32_t>(4);
    w.branch = c.take<int32_t>(1);
    w.scan_tmp = c.take<char>(scan_temp_bytes(cap));
    w.pairs = c.take<int2>(max_pairs);
}

// Xbar (values on X's slots) of one frozen step: X = X~_{t-1} with norms,
// G the symmetric gradient on the pattern of X~_t.
void run_adjoint_step(const MatView& X, const MatView& G, double tau, int branch, double* xbar, AdjWs& w,
                      hipStream_t s) {
    fill_u32(w.bitsX, (int64_t)w.nb * w.nw, 0u, s);
    fill_u32(w.bitsG, (int64_t)w.nb * w.nw, 0u, s);
    launch_occupancy(X, kOccA, w.bitsX, w.nw, nullptr, 0, 0, nullptr, s);
    launch_occupancy(G, kOccA, w.bitsG, w.nw, nullptr, 0, 0, nullptr, s);
    fill_i32(w.branch, 1, branch, s);
    launch_adj_outputs(X, w.flag, w.pos, w.oi, w.oj, &w.sc[0], w.scan_tmp, s);
    launch_adj_pairs(w.nb, w.nw, w.cap, &w.sc[0], w.oi, w.oj, w.bitsX, w.bitsG, X.map, X.norm, G.map, tau, w.cnt,
                     w.optr, &w.sc[1], w.cap_pairs, w.pairs, w.ovf, w.scan_tmp, s);
    GemmArgs g;
    g.b = X.b;
    g.nb = X.nb;
    g.oi = w.oi;
    g.oj = w.oj;
    g.optr = w.optr;
    g.pairs = w.pairs;
    g.nout = &w.sc[0];
    g.npairs = &w.sc[1];
    g.valA = G.val;
    g.valB = X.val;
    g.btrans = 1;
    g.sym = 1;
    g.map_out = X.map;
    g.val_out = xbar;
    g.mapX = G.map;
    g.valX = G.val;
    g.branch = w.branch;
    g.counters = w.counters;
    g.ovf = w.ovf;
    g.done = nullptr;
    launch_gemm_f64(g, num_cus(), s);
}

// SPAMM_WTAUFALLBACK when some step of a purification found no candidate
// threshold below its budget and ran the exact product (tau = 0); Algorithm 1
// (variant 2) always runs it and gets no warning.
int tau_fallback_status(int status, const sp2_iter_log* log, int nlog, int variant, int N) {
    if (status != SPAMM_OK || variant == 2) return status;
    for (int q = 0; q < nlog; ++q)
        if (log[q].branch >= 0 && log[q].idx >= N)
            return fail(SPAMM_WTAUFALLBACK, "iteration %d: no candidate threshold met the budget, tau = 0 (exact product)",
                        log[q].i);
    return status;
}

}  // namespace

extern "C" {

const char* spamm_last_error(void) { return g_err; }

int spamm_version(void) { return 100; }

const char* spamm_status_str(int code) {
    switch (code) {
        case SPAMM_OK: return "ok";
        case SPAMM_EINVAL: return "invalid argument";
        case SPAMM_ECAPACITY: return "capacity exceeded";
        case SPAMM_EWORKSPACE: return "workspace too small";
        case SPAMM_EHIP: return "HIP runtime error";
        case SPAMM_ENOTSUP: return "not supported";
        case SPAMM_WNOCONV: return "iteration limit reached before the stop rule";
        case SPAMM_WTAUFALLBACK: return "no candidate met the budget; exact product used";
        default: return "unknown status";
    }
}

int spamm_build_norms(spamm_bsm* X, spamm_stream_t stream) {
    int rc = check_bsm(X, "X", true);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    launch_norms(X->b, X->nslot, X->cap, X->brow, X->val, X->sq, X->sqlo, X->norm, s);
    HIP_TRY(hipGetLastError());
    return SPAMM_OK;
}

size_t spamm_sweep_workspace_bytes(int32_t nb, int32_t N) {
    if (nb < 1 || N < 1) return 0;
    Carver c(nullptr);
    SweepWs w;
    carve_sweep(c, nb, N, w);
    return c.off + 256;
}

int spamm_sweep_tau(const spamm_bsm* A, const spamm_bsm* B, const double* tau, int32_t N, const double* budget,
                    double budget_host, int32_t mode, const double* tau0_dev, double c_low, uint32_t flags,
                    double* bound_out, int32_t* idx_out, double* tau_out, void* ws, size_t ws_bytes,
                    spamm_stream_t stream) {
    int rc = check_bsm(A, "A", true);
    if (!rc) rc = check_bsm(B, "B", true);
    if (rc) return rc;
    if (A->nb != B->nb || A->b != B->b) return fail(SPAMM_EINVAL, "A and B must share n and leaf size");
    if (N < 1 || N > 1024) return fail(SPAMM_EINVAL, "N must be in [1, 1024]");
    if (!tau || !idx_out || !tau_out) return fail(SPAMM_EINVAL, "NULL output");
    if (mode == 1 && !tau0_dev) return fail(SPAMM_EINVAL, "mode 1 needs tau0");
    if (mode != 0 && mode != 1) return fail(SPAMM_EINVAL, "mode must be 0 or 1");
    const int kind = (flags & SPAMM_BOUND_FLAT) ? 1 : ((flags & SPAMM_BOUND_SUM) ? 2 : 0);
    if ((flags & SPAMM_BOUND_FLAT) && (flags & SPAMM_BOUND_SUM))
        return fail(SPAMM_EINVAL, "choose one of SPAMM_BOUND_FLAT and SPAMM_BOUND_SUM");
    if (kind != 0 && A->nb > kBoundMaxNb) return fail(SPAMM_ENOTSUP, "the leaf-level bounds support nb <= %d", kBoundMaxNb);
    size_t need = spamm_sweep_workspace_bytes(A->nb, N);
    if (!ws || ws_bytes < need) return fail(SPAMM_EWORKSPACE, "sweep needs %zu workspace bytes", need);
    hipStream_t s = (hipStream_t)stream;
    // the candidate list must be strictly decreasing and positive
    std::vector<double> th(N);
    HIP_TRY(hipMemcpyAsync(th.data(), tau, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int m = 0; m < N; ++m) {
        if (!(th[m] > 0.0) || !isfinite(th[m])) return fail(SPAMM_EINVAL, "tau[%d] must be finite and > 0", m);
        if (m > 0 && !(th[m] < th[m - 1])) return fail(SPAMM_EINVAL, "tau must be strictly decreasing");
    }
    Carver c(ws);
    SweepWs w;
    carve_sweep(c, A->nb, N, w);
    fill_i32(w.ovf, 1, 0, s);
    if (kind != 0)
        run_sweep_leaf(view(A), view(B), (flags & SPAMM_B_TRANSPOSED) ? 1 : 0, tau, N, budget, budget_host, kind,
                       mode, tau0_dev, c_low,
                       bound_out, idx_out, tau_out, w, nullptr, s);
    else
        run_sweep(view(A), view(B), (flags & SPAMM_B_TRANSPOSED) ? 1 : 0, tau, N, budget, budget_host, mode, tau0_dev,
                  c_low, bound_out, idx_out, tau_out, w, nullptr, s);
    HIP_TRY(hipGetLastError());
    if (flags & SPAMM_SYNC) {
        HIP_TRY(hipStreamSynchronize(s));
        int32_t idx = 0;
        HIP_TRY(hipMemcpy(&idx, idx_out, sizeof(idx), hipMemcpyDeviceToHost));
        if (idx >= N) return fail(SPAMM_WTAUFALLBACK, "no candidate threshold met the budget: tau = 0");
    }
    return SPAMM_OK;
}

size_t spamm_multiply_workspace_bytes(int32_t nb, int64_t max_pairs) {
    if (nb < 1) return 0;
    Carver c(nullptr);
    MulWs w;
    carve_mul(c, nb, max_pairs, w);
    c.take<uint8_t>(0);
    return c.off + 256;
}

int spamm_multiply(const spamm_bsm* A, const spamm_bsm* B, const double* tau_dev, uint32_t flags, spamm_bsm* C,
                   int64_t* kept_out, void* ws, size_t ws_bytes, spamm_stream_t stream) {
    int rc = check_bsm(A, "A", true);
    if (!rc) rc = check_bsm(B, "B", true);
    if (!rc) rc = check_bsm(C, "C", false);
    if (rc) return rc;
    if (A->nb != B->nb || A->b != B->b || C->nb != A->nb || C->b != A->b)
        return fail(SPAMM_EINVAL, "A, B and C must share n and leaf size");
    if (!tau_dev) return fail(SPAMM_EINVAL, "tau_dev is NULL");
    const int sym = (flags & SPAMM_SYMMETRIC) ? 1 : 0;
    const int btrans = (flags & SPAMM_B_TRANSPOSED) ? 1 : 0;
    // the caller's workspace fixes the pair capacity
    const size_t base = spamm_multiply_workspace_bytes(A->nb, 0);
    if (!ws || ws_bytes < base) return fail(SPAMM_EWORKSPACE, "multiply needs at least %zu workspace bytes", base);
    // pair capacity: what the workspace holds beyond the base (512 bytes slack
    // cover the alignment of the carved arrays)
    const int64_t max_pairs = ws_bytes > base + 512 ? clamp_pairs((int64_t)((ws_bytes - base - 512) / sizeof(int2))) : 0;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws);
    MulWs w;
    carve_mul(c, A->nb, max_pairs, w);
    if (c.off > ws_bytes) return fail(SPAMM_EWORKSPACE, "workspace too small");
    fill_i32(w.ovf, 1, 0, s);
    run_pairs(view(A), view(B), btrans, sym, tau_dev, nullptr, view(C), nullptr, w, nullptr, nullptr, nullptr, s);
    run_gemm(view(A), view(B), btrans, sym, view(C), nullptr, w, nullptr, nullptr, nullptr, nullptr, s);
    HIP_TRY(hipGetLastError());
    int64_t sc[3];
    int32_t ovf = 0;
    HIP_TRY(hipMemcpyAsync(sc, w.sc, sizeof(sc), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&ovf, w.ovf, sizeof(ovf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (kept_out) {
        int64_t ko[2] = {sc[0], sc[1]};
        HIP_TRY(hipMemcpyAsync(kept_out, ko, sizeof(ko), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (ovf) {
        return fail(SPAMM_ECAPACITY, "capacity exceeded: pairs %lld (cap %lld), slots %lld (cap %lld)",
                    (long long)sc[0], (long long)max_pairs, (long long)sc[2], (long long)C->cap);
    }
    return SPAMM_OK;
}

double spamm_tier_constant(int32_t precision, int32_t b) { return tier_constant(precision, b); }

size_t spamm_multiply_tiered_workspace_bytes(int32_t nb, int64_t capA, int64_t capB, int32_t b, int64_t max_pairs) {
    if (nb < 1) return 0;
    Carver c(nullptr);
    c.take<float>((size_t)capA * b * b);
    c.take<float>((size_t)capB * b * b);
    c.take<int32_t>(capA);
    c.take<int32_t>(capB);
    MulWs w;
    carve_mul(c, nb, max_pairs, w);
    return c.off + 256;
}

int spamm_multiply_tiered(const spamm_bsm* A, const spamm_bsm* B, const double* tau_dev, const double* sigma_dev,
                          uint32_t flags, spamm_bsm* C, int64_t* kept_out, void* ws, size_t ws_bytes,
                          spamm_stream_t stream) {
    int rc = check_bsm(A, "A", true);
    if (!rc) rc = check_bsm(B, "B", true);
    if (!rc) rc = check_bsm(C, "C", false);
    if (rc) return rc;
    if (A->nb != B->nb || A->b != B->b || C->nb != A->nb || C->b != A->b)
        return fail(SPAMM_EINVAL, "A, B and C must share n and leaf size");
    if (A->b > 64) return fail(SPAMM_ENOTSUP, "the precision tiers support leaf 32 and 64");
    if (!tau_dev || !sigma_dev) return fail(SPAMM_EINVAL, "tau_dev and sigma_dev are required");
    const int sym = (flags & SPAMM_SYMMETRIC) ? 1 : 0;
    const int btrans = (flags & SPAMM_B_TRANSPOSED) ? 1 : 0;
    const bool bf16 = (flags & SPAMM_TIER_BF16) != 0;
    if (bf16 && !btrans) return fail(SPAMM_ENOTSUP, "the split-BF16 tier needs SPAMM_B_TRANSPOSED");
    const size_t base = spamm_multiply_tiered_workspace_bytes(A->nb, A->cap, B->cap, A->b, 0);
    if (!ws || ws_bytes < base) return fail(SPAMM_EWORKSPACE, "tiered multiply needs at least %zu bytes", base);
    const int64_t max_pairs = ws_bytes > base + 512 ? clamp_pairs((int64_t)((ws_bytes - base - 512) / sizeof(int2))) : 0;
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws);
    float* a32 = c.take<float>((size_t)A->cap * A->b * A->b);
    float* b32 = c.take<float>((size_t)B->cap * B->b * B->b);
    int32_t* ea = c.take<int32_t>(A->cap);
    int32_t* eb = c.take<int32_t>(B->cap);
    MulWs w;
    carve_mul(c, A->nb, max_pairs, w);
    if (c.off > ws_bytes) return fail(SPAMM_EWORKSPACE, "workspace too small");
    fill_i32(w.ovf, 1, 0, s);
    uint16_t* a16 = reinterpret_cast<uint16_t*>(a32);
    uint16_t* b16 = reinterpret_cast<uint16_t*>(b32);
    if (bf16) {
        launch_to_bf16x2(A->b, A->nslot, A->cap, A->brow, A->val, a16, ea, nullptr, s);
        launch_to_bf16x2(B->b, B->nslot, B->cap, B->brow, B->val, b16, eb, nullptr, s);
    } else {
        // the ring kernel (B given transposed) reads rotated rows, the other path plain blocks
        launch_to_f32(A->b, A->nslot, A->cap, A->brow, A->val, a32, btrans, nullptr, s);
        launch_to_f32(B->b, B->nslot, B->cap, B->brow, B->val, b32, btrans, nullptr, s);
    }
    run_pairs(view(A), view(B), btrans, sym, tau_dev, sigma_dev, view(C), nullptr, w, nullptr, nullptr, nullptr, s,
              nullptr, (flags & SPAMM_TIER_BF16) ? 0.0 : kFp32TierNormMin);
    run_gemm(view(A), view(B), btrans, sym, view(C), nullptr, w, nullptr, nullptr, nullptr, nullptr, s,
             bf16 ? nullptr : a32, bf16 ? nullptr : b32, nullptr, nullptr, bf16 ? a16 : nullptr, bf16 ? b16 : nullptr,
             bf16 ? ea : nullptr, bf16 ? eb : nullptr);
    HIP_TRY(hipGetLastError());
    int64_t sc[4];
    int32_t ovf = 0;
    HIP_TRY(hipMemcpyAsync(sc, w.sc, sizeof(sc), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&ovf, w.ovf, sizeof(ovf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (kept_out) {
        int64_t ko[3] = {sc[0], sc[1], sc[3]};
        HIP_TRY(hipMemcpyAsync(kept_out, ko, sizeof(ko), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (ovf) return fail(SPAMM_ECAPACITY, "capacity exceeded (pairs %lld of %lld)", (long long)sc[0], (long long)max_pairs);
    return SPAMM_OK;
}

size_t spamm_truncate_workspace_bytes(int64_t cap) { return trunc_temp_bytes(cap) + 64 + 512; }

int spamm_truncate(spamm_bsm* X, double delta, uint32_t flags, double* removed_out, void* ws, size_t ws_bytes,
                   spamm_stream_t stream) {
    int rc = check_bsm(X, "X", true);
    if (rc) return rc;
    if (!(delta >= 0.0) || !isfinite(delta)) return fail(SPAMM_EINVAL, "delta must be finite and >= 0");
    size_t need = spamm_truncate_workspace_bytes(X->cap);
    if (!ws || ws_bytes < need) return fail(SPAMM_EWORKSPACE, "truncate needs %zu workspace bytes", need);
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws);
    void* tmp = c.take<char>(trunc_temp_bytes(X->cap));
    int64_t* stats = c.take<int64_t>(4);
    int32_t* ovf = c.take<int32_t>(4);
    fill_i32(ovf, 1, 0, s);
    launch_truncate(view(X), nullptr, delta, 1.0, tmp, X->cap, stats, ovf, nullptr, s);
    if (removed_out) hipLaunchKernelGGL(k_trunc_report, dim3(1), dim3(1), 0, s, stats, nullptr, delta, 1.0, removed_out);
    HIP_TRY(hipGetLastError());
    if (flags & SPAMM_SYNC) HIP_TRY(hipStreamSynchronize(s));
    return SPAMM_OK;
}

int64_t spamm_truncate_noalloc_max_cap(void) { return trunc_noalloc_max_cap(); }

int spamm_truncate_noalloc(spamm_bsm* X, double delta, uint32_t flags, double* removed_out, spamm_stream_t stream) {
    int rc = check_bsm(X, "X", true);
    if (rc) return rc;
    if (!(delta >= 0.0) || !isfinite(delta)) return fail(SPAMM_EINVAL, "delta must be finite and >= 0");
    if (X->cap > trunc_noalloc_max_cap())
        return fail(SPAMM_EINVAL, "spamm_truncate_noalloc: capacity %lld exceeds its limit of %lld slots",
                    (long long)X->cap, (long long)trunc_noalloc_max_cap());
    TruncNoallocScratch sc;
    HIP_TRY(trunc_noalloc_scratch(&sc));
    hipStream_t s = (hipStream_t)stream;
    fill_i32(sc.ovf, 1, 0, s);
    launch_truncate(view(X), nullptr, delta, 1.0, sc.temp, X->cap, sc.stats, sc.ovf, nullptr, s);
    if (removed_out)
        hipLaunchKernelGGL(k_trunc_report, dim3(1), dim3(1), 0, s, sc.stats, nullptr, delta, 1.0, removed_out);
    HIP_TRY(hipGetLastError());
    if (flags & SPAMM_SYNC) HIP_TRY(hipStreamSynchronize(s));
    return SPAMM_OK;
}

size_t purify_sp2_workspace_bytes(int32_t nb, int32_t b, int32_t N, int64_t cap_blocks, int64_t max_pairs,
                                  int32_t tape_steps, int32_t precision) {
    if (nb < 1 || N < 1 || cap_blocks < 1) return 0;
    Carver c(nullptr);
    Sp2Ws w;
    carve_sp2(c, nb, b, N, cap_blocks, max_pairs, tape_steps, w, precision);
    return c.off + 256;
}

int purify_sp2_tape_view(void* ws, int32_t nb, int32_t b, int32_t N, int64_t cap_blocks, int64_t max_pairs,
                         int32_t tape_steps, int32_t step, spamm_bsm* out) {
    if (!ws || !out || nb < 1 || N < 1 || cap_blocks < 1) return fail(SPAMM_EINVAL, "bad tape view arguments");
    if (step < 0 || step > tape_steps) return fail(SPAMM_EINVAL, "tape step out of range");
    Carver c(ws);
    Sp2Ws w;
    carve_sp2(c, nb, b, N, cap_blocks, max_pairs, tape_steps, w);
    *out = w.tape[step];
    return SPAMM_OK;
}

// purify_sp2 with an extra limit: the host loop stops after max_steps
// steps (status SPAMM_WNOCONV) while delta_i still follows p->n_max
static int purify_run(const spamm_bsm* F, const sp2_params* p, spamm_bsm* D, sp2_iter_log* log, int32_t* nlog_out,
                      void* ws, size_t ws_bytes, spamm_stream_t stream, int max_steps) {
    if (!log || !nlog_out) return fail(SPAMM_EINVAL, "NULL argument");
    int rc = check_sp2(F, p, D);
    if (rc) return rc;
    const bool have_gap = !isnan(p->homo) && !isnan(p->lumo);
    const bool tiered = p->precision != 0;
    const double c_low = tier_constant(p->precision, F->b);
    const int nb = F->nb, b = F->b;
    // keep_tape: 0 none, 1 every iterate, k > 1 every k-th iterate (checkpoints)
    const int every = p->keep_tape;
    const int tape_steps = every == 1 ? p->n_max : (every > 1 ? p->n_max / every : 0);
    // internal capacity: whatever the workspace holds (the binding sizes it)
    int64_t cap = 0;
    {
        // find the largest cap with the given pair capacity that fits: the
        // binding passes the same cap/pairs it queried with, encoded in D->cap
        cap = D->cap;
    }
    int64_t max_pairs = 0;
    {
        size_t base = purify_sp2_workspace_bytes(nb, b, p->N, cap, 0, tape_steps, p->precision);
        if (!ws || ws_bytes < base) return fail(SPAMM_EWORKSPACE, "purify needs at least %zu workspace bytes", base);
        max_pairs = ws_bytes > base + 512 ? clamp_pairs((int64_t)((ws_bytes - base - 512) / sizeof(int2))) : 0;
    }
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws);
    Sp2Ws w;
    carve_sp2(c, nb, b, p->N, cap, max_pairs, tape_steps, w, p->precision);
    if (c.off > ws_bytes) return fail(SPAMM_EWORKSPACE, "workspace too small");
    // ev[0..5]: phase times (host loop), ev[6]: start of the device loop,
    // ev[8]/ev[9]: fork and join of the split-BF16 copy's side stream
    hipEvent_t ev[10] = {};
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard() {
            for (int q = 0; q < 10; ++q)
                if (e[q]) (void)hipEventDestroy(e[q]);
        }
    } guard{ev};
    for (int q = 0; q < 8; ++q) HIP_TRY(hipEventCreate(&ev[q]));
    for (int q = 8; q < 10; ++q) HIP_TRY(hipEventCreateWithFlags(&ev[q], hipEventDisableTiming));
    // (host-driven loop only: on this ROCm a graph captured with a fork and
    // a join was seen to keep the device memory of the buffers it had used
    // unavailable after they were freed, so a captured step stays on one
    // stream)
    hipStream_t side = nullptr;
    if (p->precision == 2 && p->graph_steps <= 0) HIP_TRY(kept_stream(1, &side));
    // the side copy runs with one workgroup per CU, leaving the rest of each
    // CU to the sweeps' kernels beside it (more workgroups made the step
    // slower at n = 16384 and 65536)
    const int side_wg = num_cus();

    Sp2Ctl hc;
    memset(&hc, 0, sizeof(hc));
    fill_i32(w.mw.ovf, 1, 0, s);
    fill_i32(w.sw.ovf, 1, 0, s);
    fill_i64(w.tstats, 4, 0, s);  // stays 0 when no step truncates (Algorithm 4)
    launch_traces_init(w.trace_tmp, s);

    // X_0 and its first truncation: the spectral bounds and the slot count
    // of F in one read-back, then the capacity check before X_0 is written
    // (the device-driven loop reads nothing back: the control block, with the
    // mapped gap and delta_0, is set up by a kernel from the bounds on the
    // device; the host loop reads the bounds and keeps the gap on the host)
    const double tb_scale = p->variant == 0 ? 0.5 : 1.0;
    const bool device_loop = p->graph_steps > 0;
    MatView Fv = view(F);
    MatView X0 = view(&w.X[0]);
    launch_gersch(Fv, w.rowtmp, w.lam, s);
    double lam[2] = {0.0, 0.0};
    int32_t nf = 0;
    const bool check_cap = cap < (int64_t)nb * nb;  // nb^2 slots always hold X_0
    if (!device_loop) HIP_TRY(hipMemcpyAsync(lam, w.lam, sizeof(lam), hipMemcpyDeviceToHost, s));
    if (check_cap) HIP_TRY(hipMemcpyAsync(&nf, F->nslot, sizeof(nf), hipMemcpyDeviceToHost, s));
    if (!device_loop || check_cap) HIP_TRY(hipStreamSynchronize(s));
    if (check_cap && (int64_t)nf + nb > cap)
        return fail(SPAMM_ECAPACITY, "D->cap must be at least min(nslot(F) + nb, nb^2)");
    double xh = NAN, xl = NAN;
    if (device_loop) {
        hc.eps = p->eps;
        hc.homo = p->homo;
        hc.lumo = p->lumo;
        hc.delta_const = p->delta_const;
        hc.e_tol = p->e_tol;
        hc.n_occ = p->n_occ;
        hc.n_max = p->n_max;
        hc.variant = p->variant;
        hc.N = p->N;
        hc.n_e = 0;
        hc.done = 0;
        hc.nlog = 0;
        hc.status = SPAMM_OK;
        hc.tiered = tiered ? 1 : 0;
        hc.have_gap = have_gap ? 1 : 0;
        hc.tier_split = p->tier_split;
        hc.trunc_scale = tb_scale;
        launch_sp2_init(hc, w.lam, w.ctl, s);
    } else {
        const double W = lam[1] - lam[0];
        xh = have_gap ? (lam[1] - p->homo) / W : NAN;
        xl = have_gap ? (lam[1] - p->lumo) / W : NAN;
        hc.delta = step_delta(p, xh - xl);
        HIP_TRY(hipMemcpyAsync(w.ctl, &hc, sizeof(hc), hipMemcpyHostToDevice, s));
    }
    launch_x0(Fv, w.lam, X0, w.dflag, w.dpos, w.mw.scan_tmp, w.dcount, s);
    launch_norms(b, X0.nslot, X0.cap, X0.brow, X0.val, X0.sq, X0.sqlo, X0.norm, s);
    if (p->variant != 1) launch_truncate(X0, &w.ctl->delta, 0.0, 1.0, w.trunc_tmp, cap, w.tstats, w.mw.ovf, nullptr, s);
    const bool full_tape = every == 1;
    if (every >= 1) {
        // tape[0] = X~_0
        const int rcc = copy_mat(w.tape[0], w.X[0], cap, s);
        if (rcc) return rcc;
    }

    // One purification step on the device, X~_{i-1} (xv) -> X~_i (nv), with
    // every decision read from the control block: the threshold sweep (and
    // the low-precision limit), kept pairs and output pattern, the leaf
    // products with the combine fused, block norms, truncation.  done: the
    // device stop flag (graph mode), null in the host loop.  evs: phase
    // events (host loop only).
    // FP32 tier (one system): the FP32 copy of X~_{i-1} is f32buf[par] and the
    // product writes the copy of X~_i into f32buf[1 - par] (par: the step's
    // parity), so no conversion pass runs inside the loop
    float* f32buf[2] = {w.x32, w.x32n};
    const bool f32_fused = p->precision == 1 && w.x32n != nullptr;
    if (f32_fused) launch_to_f32(b, X0.nslot, X0.cap, X0.brow, X0.val, f32buf[0], 1, nullptr, s);  // X~_0
    auto enqueue_step = [&](const MatView& xv, const MatView& nv, int par, const int32_t* done, hipEvent_t* evs,
                            hipStream_t st) -> int {
        if (evs) HIP_TRY(hipEventRecord(evs[0], st));
        // split-BF16 tier, host-driven loop: the copies of X~_i (an HBM-bound
        // pass) run on the side stream beside the occupancy pass and the two
        // sweeps, which read only the block pattern and norms; joined before
        // the products
        if (side) {
            HIP_TRY(hipEventRecord(ev[8], st));
            HIP_TRY(hipStreamWaitEvent(side, ev[8], 0));
            launch_to_bf16x2(b, xv.nslot, xv.cap, xv.brow, xv.val, reinterpret_cast<uint16_t*>(w.x32), w.xexp, done,
                             side, side_wg);
            HIP_TRY(hipEventRecord(ev[9], side));
        }
        // the iterate's occupancy, shared by the sweeps and the kept pairs
        const SymOcc occ = build_sym_occ(xv, w.mw.bitsA, w.mw.nw, w.sw.tA, w.sw.T, w.sw.l0, done, st, &w.sw);
        if (p->variant != 2 && p->bound_kind != 0)
            run_sweep_leaf(xv, xv, 1, p->tau, p->N, &w.ctl->budget_skip, 0.0, p->bound_kind, 0, nullptr, 0.0,
                           w.bound, &w.ctl->idx,
                           &w.ctl->tau, w.sw, done, st, &occ);
        else if (p->variant != 2)
            run_sweep(xv, xv, 1, p->tau, p->N, &w.ctl->budget_skip, 0.0, 0, nullptr, 0.0, w.bound, &w.ctl->idx,
                      &w.ctl->tau, w.sw, done, st, &occ);
        if (tiered) {
            // largest low-precision limit whose bound (skipped p plus c_low p for the low
            // tier) stays below the whole product budget
            if (p->bound_kind != 0)
                run_sweep_leaf(xv, xv, 1, p->tau, p->N, &w.ctl->budget, 0.0, p->bound_kind, 1, &w.ctl->tau, c_low,
                               w.bound2, &w.ctl->sidx, &w.ctl->sigma, w.sw, done, st, &occ);
            else
                run_sweep(xv, xv, 1, p->tau, p->N, &w.ctl->budget, 0.0, 1, &w.ctl->tau, c_low, w.bound2,
                          &w.ctl->sidx, &w.ctl->sigma, w.sw, done, st, &occ);
            if (p->precision == 2 && !side)
                launch_to_bf16x2(b, xv.nslot, xv.cap, xv.brow, xv.val, reinterpret_cast<uint16_t*>(w.x32), w.xexp,
                                 done, st);
            else if (p->precision == 1 && !f32_fused)
                launch_to_f32(b, xv.nslot, xv.cap, xv.brow, xv.val, w.x32, 1, done, st);
        }
        if (side) HIP_TRY(hipStreamWaitEvent(st, ev[9], 0));
        if (evs) HIP_TRY(hipEventRecord(evs[1], st));
        // kept pairs, output pattern and the leaf products (combined with X),
        // with the block norms of the new iterate
        NormOut step_norms;
        step_norms.sq = nv.sq;
        step_norms.sqlo = nv.sqlo;
        step_norms.nrm = nv.norm;
        step_norms.recheck = w.recheck;
        step_norms.nrecheck = &w.mw.counters[8];
        run_pairs(xv, xv, 1, 1, &w.ctl->tau, tiered ? &w.ctl->sigma : nullptr, nv, w.fromc, w.mw, xv.map,
                  &w.ctl->branch, done, st, &occ, p->precision == 1 ? kFp32TierNormMin : 0.0);
        // evs[2]/evs[3] bracket the product kernel alone
        const uint16_t* x16 = p->precision == 2 ? reinterpret_cast<const uint16_t*>(w.x32) : nullptr;
        const float* x32 = p->precision == 1 ? (f32_fused ? f32buf[par] : w.x32) : nullptr;
        const int32_t* xexp = p->precision == 2 ? w.xexp : nullptr;
        const int rg = run_gemm(xv, xv, 1, 1, nv, w.fromc, w.mw, xv.map, xv.val, &w.ctl->branch, done, st, x32, x32,
                                evs ? evs[2] : nullptr, evs ? evs[3] : nullptr, x16, x16, xexp, xexp, step_norms,
                                f32_fused ? f32buf[1 - par] : nullptr);
        if (rg) return fail(SPAMM_EINVAL, "fused block norms or FP32 copies need the transposed-B product");
        launch_norms_listed(b, w.recheck, &w.mw.counters[8], nv.cap, nv.brow, nv.val, nv.sq, nv.sqlo, nv.norm, st,
                            done);
        if (evs) HIP_TRY(hipEventRecord(evs[4], st));
        if (p->variant != 1)
            launch_truncate(nv, &w.ctl->delta, 0.0, tb_scale, w.trunc_tmp, cap, w.tstats, w.mw.ovf, done, st);
        if (evs) HIP_TRY(hipEventRecord(evs[5], st));
        HIP_TRY(hipGetLastError());
        return SPAMM_OK;
    };

    int cur = 0;
    int nlog = 0;
    int status = SPAMM_OK;
    if (p->graph_steps > 0) {
        // ---- device-driven loop: two steps (X0 -> X1 -> X0) captured once,
        // replayed until the control step sets done (the control block was
        // set up with X_0) ----
        (void)num_cus();  // device properties are read once, outside the capture
        GraphGuard gg;
        HIP_TRY(capture_stream(&gg.cs));
        HIP_TRY(hipEventRecord(ev[6], s));
        HIP_TRY(hipStreamWaitEvent(gg.cs, ev[6], 0));
        HIP_TRY(hipStreamBeginCapture(gg.cs, hipStreamCaptureModeThreadLocal));
        int rc_cap = SPAMM_OK;
        for (int q = 0; q < 2 && rc_cap == SPAMM_OK; ++q) {
            MatView xv = view(&w.X[q]);
            MatView nv = view(&w.X[1 - q]);
            launch_traces(xv.nslot, xv.cap, b, F->n, xv.brow, xv.bcol, xv.val, xv.sq, xv.sqlo, w.trace_tmp,
                          w.trace_out, &w.ctl->done, gg.cs, control_tail(w));
            rc_cap = enqueue_step(xv, nv, q, &w.ctl->done, nullptr, gg.cs);
        }
        hipError_t ec = hipStreamEndCapture(gg.cs, &gg.g);
        if (rc_cap != SPAMM_OK) return rc_cap;
        if (ec != hipSuccess) return fail(SPAMM_EHIP, "graph capture: %s", hipGetErrorString(ec));
        HIP_TRY(hipGraphInstantiate(&gg.ge, gg.g, nullptr, nullptr, 0));
        const int per_poll = std::max(1, (p->graph_steps + 1) / 2);
        const int max_replays = p->n_max / 2 + 2;  // n_max + 4 control steps: the stop always fires
        int32_t done = 0;
        for (int r = 0; r < max_replays && !done;) {
            for (int q = 0; q < per_poll && r < max_replays; ++q, ++r) HIP_TRY(hipGraphLaunch(gg.ge, gg.cs));
            HIP_TRY(hipMemcpyAsync(&done, &w.ctl->done, sizeof(done), hipMemcpyDeviceToHost, gg.cs));
            HIP_TRY(hipStreamSynchronize(gg.cs));
        }
        Sp2Ctl cs;
        int64_t msc[4];
        HIP_TRY(hipMemcpyAsync(&cs, w.ctl, sizeof(cs), hipMemcpyDeviceToHost, gg.cs));
        HIP_TRY(hipMemcpyAsync(msc, w.mw.sc, sizeof(msc), hipMemcpyDeviceToHost, gg.cs));
        HIP_TRY(hipStreamSynchronize(gg.cs));
        if (!done) return fail(SPAMM_EHIP, "device loop did not reach its stop");
        nlog = cs.nlog;
        if (nlog > 0)
            HIP_TRY(hipMemcpy(log, w.dlog, sizeof(sp2_iter_log) * (size_t)nlog, hipMemcpyDeviceToHost));
        if (cs.status == SPAMM_ECAPACITY) {
            status = fail(SPAMM_ECAPACITY, "capacity exceeded in iteration %d (pairs %lld of %lld)", nlog,
                          (long long)msc[0], (long long)max_pairs);
        } else {
            status = cs.status;
        }
        cur = (nlog - 1) & 1;
    } else {
        std::vector<double> e_hist;
        // the step's read-back lands in host-mapped memory, gathered by one kernel
        struct PinnedStatus {
            Sp2HostStatus* h = nullptr;
            ~PinnedStatus() {
                if (h) (void)hipHostFree(h);
            }
        } ps;
        HIP_TRY(hipHostMalloc((void**)&ps.h, sizeof(Sp2HostStatus), hipHostMallocMapped | hipHostMallocCoherent));
        Sp2HostStatus* hs_dev = nullptr;
        HIP_TRY(hipHostGetDevicePointer((void**)&hs_dev, ps.h, 0));
        for (int it = 1;; ++it) {
            spamm_bsm* Xc = full_tape ? &w.tape[it - 1] : &w.X[cur];
            spamm_bsm* Xn = full_tape ? (it <= tape_steps ? &w.tape[it] : nullptr) : &w.X[1 - cur];
            MatView xv = view(Xc);
            TraceTail tail;
            tail.hs = hs_dev;
            tail.ctl_read = w.ctl;
            tail.msc = w.mw.sc;
            tail.ts = w.tstats;
            tail.ovf_mul = w.mw.ovf;
            tail.ovf_sweep = w.sw.ovf;
            launch_traces(xv.nslot, xv.cap, b, F->n, xv.brow, xv.bcol, xv.val, xv.sq, xv.sqlo, w.trace_tmp,
                          w.trace_out, nullptr, s, tail);
            double tr[4];
            int64_t msc[4], ts[3];
            int32_t ovf[2];
            Sp2Ctl cs;
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipStreamSynchronize(s));
            memcpy(tr, ps.h->tr, sizeof(tr));
            memcpy(msc, ps.h->msc, sizeof(msc));
            memcpy(ts, ps.h->ts, sizeof(ts));
            memcpy(ovf, ps.h->ovf, sizeof(ovf));
            memcpy(&cs, &ps.h->ctl, sizeof(cs));
            if (ovf[0] || ovf[1]) {
                status = fail(SPAMM_ECAPACITY, "capacity exceeded in iteration %d (flags %d/%d; pairs %lld of %lld)",
                              it - 1, ovf[0], ovf[1], (long long)msc[0], (long long)max_pairs);
                break;
            }
            if (nlog > 0) {
                sp2_iter_log& L = log[nlog - 1];
                L.idx = cs.idx;
                L.tau = cs.tau;
                L.npairs = msc[0];
                L.nout = msc[1];
                L.nslot_hat = msc[2];
                L.removed_units = ts[0];
                L.removed_fro2 = (double)ts[1] * trunc_quantum(L.delta * tb_scale);
                L.nslot_kept = msc[2] - ts[2];  // blocks of X~: those of X^ minus the removed ones
                L.npairs_low = tiered ? msc[3] : 0;
                L.sigma = cs.sigma;
                L.sidx = cs.sidx;
                // phase times (0 when an interval cannot be read)
                auto elapsed = [](hipEvent_t a, hipEvent_t z) -> float {
                    float ms = 0.f;
                    return hipEventElapsedTime(&ms, a, z) == hipSuccess ? ms : 0.f;
                };
                L.ms_sweep = elapsed(ev[0], ev[1]);
                L.ms_pairs = elapsed(ev[1], ev[2]);
                L.ms_gemm = elapsed(ev[2], ev[3]);
                L.ms_norms = elapsed(ev[3], ev[4]);
                L.ms_trunc = elapsed(ev[4], ev[5]);
                L.ms_total = elapsed(ev[0], ev[5]);
            }
            const double t1 = tr[0], t2 = tr[2];
            const double e = dd_diff(tr[0], tr[1], tr[2], tr[3]);
            e_hist.push_back(e);
            sp2_iter_log& L = log[nlog++];
            memset(&L, 0, sizeof(L));
            L.i = it;
            L.t1 = t1;
            L.t2 = t2;
            L.e = e;
            L.branch = -1;
            const bool stop = should_stop(e_hist, p->e_tol);
            if (stop || it > p->n_max || Xn == nullptr || it > max_steps) {
                L.stop = stop ? 1 : 2;
                if (!stop) status = SPAMM_WNOCONV;
                break;
            }
            const int br = choose_branch(t1, t2, p->n_occ);
            if (have_gap) {
                xh = map_gap(xh, br);
                xl = map_gap(xl, br);
            }
            const double delta = step_delta(p, xh - xl);
            L.branch = br;
            L.delta = delta;
            hc.branch = br;
            hc.delta = delta;
            hc.budget = p->variant == 0 ? delta / 2.0 : delta;
            hc.budget_skip = tiered ? p->tier_split * hc.budget : hc.budget;
            hc.tau = 0.0;
            hc.idx = p->N;
            hc.sigma = 0.0;
            hc.sidx = p->N;
            ps.h->ctl_in = hc;  // read by the upload kernel, launched after this store
            std::atomic_thread_fence(std::memory_order_seq_cst);
            launch_ctl_upload(&hs_dev->ctl_in, w.ctl, s);
            const int rc_step = enqueue_step(xv, view(Xn), (it - 1) & 1, nullptr, ev, s);
            if (rc_step != SPAMM_OK) return rc_step;
            if (every > 1 && it % every == 0 && it / every <= tape_steps) {
                const int rcc = copy_mat(w.tape[it / every], *Xn, cap, s);  // checkpoint X~_it
                if (rcc) return rcc;
            }
            cur = 1 - cur;
        }
    }
    // final: copy the last iterate into D
    if (status >= 0) {
        spamm_bsm* Xf = full_tape ? &w.tape[nlog - 1] : &w.X[cur];
        const int rcc = copy_mat(*D, *Xf, cap, s);
        if (rcc) return rcc;
        HIP_TRY(hipStreamSynchronize(s));
    }
    *nlog_out = nlog;
    return tau_fallback_status(status, log, nlog, p->variant, p->N);
}

int purify_sp2(const spamm_bsm* F, const sp2_params* p, spamm_bsm* D, sp2_iter_log* log, int32_t* nlog_out, void* ws,
               size_t ws_bytes, spamm_stream_t stream) {
    return purify_run(F, p, D, log, nlog_out, ws, ws_bytes, stream, 1 << 30);
}

size_t spamm_adjoint_step_workspace_bytes(int32_t nb, int64_t cap_blocks, int64_t max_pairs) {
    if (nb < 1 || cap_blocks < 1 || max_pairs < 0) return 0;
    Carver c(nullptr);
    AdjWs w;
    carve_adj(c, nb, cap_blocks, max_pairs, w);
    return c.off + 256;
}

int spamm_adjoint_step(const spamm_bsm* X, const spamm_bsm* G, double tau, int32_t branch, double* xbar_val,
                       int64_t* counts_out, void* ws, size_t ws_bytes, spamm_stream_t stream) {
    int rc = check_bsm(X, "X", true);
    if (!rc) rc = check_bsm(G, "G", false);
    if (rc) return rc;
    if (X->nb != G->nb || X->b != G->b) return fail(SPAMM_EINVAL, "X and G must have the same block grid");
    if (!(tau >= 0.0)) return fail(SPAMM_EINVAL, "tau must be >= 0");
    if (branch != 0 && branch != 1) return fail(SPAMM_EINVAL, "branch must be 0 or 1");
    if (!xbar_val) return fail(SPAMM_EINVAL, "xbar_val is NULL");
    const int64_t cap = X->cap;
    const size_t base = spamm_adjoint_step_workspace_bytes(X->nb, cap, 0);
    if (!ws || ws_bytes < base + 512) return fail(SPAMM_EWORKSPACE, "adjoint step needs more than %zu workspace bytes", base);
    const int64_t max_pairs = clamp_pairs((int64_t)((ws_bytes - base - 512) / sizeof(int2)));
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws);
    AdjWs w;
    carve_adj(c, X->nb, cap, max_pairs, w);
    if (c.off > ws_bytes) return fail(SPAMM_EWORKSPACE, "workspace too small");
    fill_i32(w.ovf, 1, 0, s);
    run_adjoint_step(view(X), view(G), tau, branch, xbar_val, w, s);
    if (counts_out) HIP_TRY(hipMemcpyAsync(counts_out, w.sc, 2 * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    int32_t ovf = 0;
    int64_t sc[2];
    HIP_TRY(hipMemcpyAsync(&ovf, w.ovf, sizeof(ovf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(sc, w.sc, sizeof(sc), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    if (ovf) return fail(SPAMM_ECAPACITY, "adjoint step needs %lld pairs, workspace holds %lld", (long long)sc[1],
                         (long long)max_pairs);
    return SPAMM_OK;
}

}  // extern "C"

namespace {

// workspace of the whole-run adjoint: two gradient buffers, the Gerschgorin
// scratch, one reverse step, and with checkpoints (tape_every > 1) the
// buffers and scratch of the forward recomputation of one segment
struct AdjRunWs {
    double* gbuf[2];
    double* rowtmp;
    double* lam;
    AdjWs aw;
    std::vector<spamm_bsm> seg;
    MulWs mw;
    uint8_t* fromc;
    void* trunc_tmp;
    int64_t* tstats;
    Sp2Ctl* ctl;
};

void carve_adj_run(Carver& c, int nb, int b, int64_t cap, int64_t max_pairs, int every, AdjRunWs& w) {
    w.gbuf[0] = c.take<double>((size_t)cap * b * b);
    w.gbuf[1] = c.take<double>((size_t)cap * b * b);
    w.rowtmp = c.take<double>(2 * (size_t)nb * b);
    w.lam = c.take<double>(2);
    carve_adj(c, nb, cap, max_pairs, w.aw);
    w.seg.clear();
    if (every > 1) {
        w.seg.resize(every - 1);
        for (auto& m : w.seg) carve_mat(c, (int64_t)nb * b, b, cap, m);
        carve_mul(c, nb, max_pairs, w.mw);
        w.fromc = c.take<uint8_t>(cap);
        w.trunc_tmp = c.take<char>(trunc_temp_bytes(cap));
        w.tstats = c.take<int64_t>(4);
        w.ctl = c.take<Sp2Ctl>(1);
    }
}

}  // namespace

extern "C" {

size_t purify_sp2_adjoint_workspace_bytes(int32_t nb, int32_t b, int64_t cap_blocks, int64_t max_pairs,
                                          int32_t tape_every) {
    if (nb < 1 || cap_blocks < 1 || max_pairs < 0 || tape_every < 1) return 0;
    Carver c(nullptr);
    AdjRunWs w;
    carve_adj_run(c, nb, b, cap_blocks, max_pairs, tape_every, w);
    return c.off + 256;
}

int purify_sp2_adjoint(const spamm_bsm* F, const sp2_params* p, const spamm_bsm* tape, int32_t ntape,
                       int32_t tape_every, const spamm_bsm* D, const sp2_iter_log* log, int32_t nlog,
                       const double* dbar_val, double* fbar_val, void* ws, size_t ws_bytes, spamm_stream_t stream) {
    int rc = check_bsm(F, "F", false);
    if (rc) return rc;
    if (!p || !tape || ntape < 1 || !log || nlog < 1 || !dbar_val || !fbar_val)
        return fail(SPAMM_EINVAL, "NULL or empty argument");
    if (tape_every < 1) return fail(SPAMM_EINVAL, "tape_every must be >= 1");
    const int T = nlog - 1;  // steps of the recorded run
    const int every = tape_every;
    if (every == 1 && ntape != nlog)
        return fail(SPAMM_EINVAL, "a full tape of a run with %d records has %d entries, not %d", nlog, nlog, ntape);
    if (every > 1 && ntape < T / every + 1)
        return fail(SPAMM_EINVAL, "%d checkpoints every %d steps do not cover %d steps", ntape, every, T);
    if (every > 1 && !D) return fail(SPAMM_EINVAL, "D is required with checkpoints");
    if (every > 1 && p->precision != 0)
        return fail(SPAMM_ENOTSUP, "recomputation from checkpoints supports FP64 runs (use a full tape)");
    const int nb = F->nb, b = F->b;
    int64_t cap = 0;
    for (int t = 0; t < ntape; ++t) {
        rc = check_bsm(&tape[t], "tape entry", true);
        if (rc) return rc;
        // tape entries carry the padded size nb * b
        if (tape[t].nb != nb || tape[t].b != b) return fail(SPAMM_EINVAL, "tape entry %d does not match F", t);
        cap = std::max<int64_t>(cap, tape[t].cap);
    }
    if (D) {
        rc = check_bsm(D, "D", true);
        if (rc) return rc;
        if (D->nb != nb || D->b != b || D->cap > cap) return fail(SPAMM_EINVAL, "D does not match the tape");
    }
    for (int t = 1; t <= T; ++t)
        if (log[t - 1].branch != 0 && log[t - 1].branch != 1)
            return fail(SPAMM_EINVAL, "log record %d is not a step", t - 1);
    const size_t base = purify_sp2_adjoint_workspace_bytes(nb, b, cap, 0, every);
    if (!ws || ws_bytes < base + 512) return fail(SPAMM_EWORKSPACE, "adjoint needs more than %zu workspace bytes", base);
    // the pair lists of the reverse step and (with checkpoints) of the
    // recomputation share what is left of the workspace
    const int64_t per_pair = every > 1 ? 2 * (int64_t)sizeof(int2) : (int64_t)sizeof(int2);
    const int64_t max_pairs = clamp_pairs((int64_t)((ws_bytes - base - 512) / per_pair));
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws);
    AdjRunWs w;
    carve_adj_run(c, nb, b, cap, max_pairs, every, w);
    if (c.off > ws_bytes) return fail(SPAMM_EWORKSPACE, "workspace too small");
    const double tb_scale = p->variant == 0 ? 0.5 : 1.0;

    fill_i32(w.aw.ovf, 1, 0, s);
    if (every > 1) fill_i32(w.mw.ovf, 1, 0, s);
    // X~_t of the recorded run: tape entry, recomputed segment buffer, or D
    int seg0 = -1;  // first step of the segment held in w.seg (X~_{seg0+1} ..)
    auto iterate = [&](int t) -> const spamm_bsm* {
        if (every == 1) return &tape[t];
        if (t == T) return D;
        if (t % every == 0) return &tape[t / every];
        return &w.seg[t - seg0 - 1];
    };
    // recompute X~_{t0+1} .. X~_{t1-1} from the checkpoint X~_{t0} with the
    // recorded decisions: the forward's own kernels, so bit-identical
    auto recompute = [&](int t0, int t1) -> int {
        seg0 = t0;
        for (int t = t0 + 1; t < t1; ++t) {
            const spamm_bsm* Xc = (t - 1 == t0) ? &tape[t0 / every] : &w.seg[t - 1 - t0 - 1];
            const spamm_bsm* Xn = &w.seg[t - t0 - 1];
            Sp2Ctl hc;
            memset(&hc, 0, sizeof(hc));
            hc.tau = log[t - 1].tau;
            hc.branch = log[t - 1].branch;
            hc.delta = log[t - 1].delta;
            HIP_TRY(hipMemcpyAsync(w.ctl, &hc, sizeof(hc), hipMemcpyHostToDevice, s));
            MatView xv = view(Xc), nv = view(Xn);
            run_pairs(xv, xv, 1, 1, &w.ctl->tau, nullptr, nv, w.fromc, w.mw, xv.map, &w.ctl->branch, nullptr, s);
            run_gemm(xv, xv, 1, 1, nv, w.fromc, w.mw, xv.map, xv.val, &w.ctl->branch, nullptr, s);
            launch_norms(b, nv.nslot, nv.cap, nv.brow, nv.val, nv.sq, nv.sqlo, nv.norm, s);
            if (p->variant != 1)
                launch_truncate(nv, &w.ctl->delta, 0.0, tb_scale, w.trunc_tmp, cap, w.tstats, w.mw.ovf, nullptr, s);
            // the host copy of hc must outlive the enqueued copy
            HIP_TRY(hipStreamSynchronize(s));
        }
        return SPAMM_OK;
    };

    // gradient of the last iterate, symmetrised
    launch_sym_half(view(iterate(T)), dbar_val, w.gbuf[0], s);
    int cur = 0;
    int t = T;
    while (t >= 1) {
        // segment [t0, t]: t0 the checkpoint at or below t - 1
        const int t0 = every == 1 ? t - 1 : ((t - 1) / every) * every;
        if (every > 1) {
            rc = recompute(t0, t);
            if (rc) return rc;
        }
        for (; t > t0; --t) {
            MatView gv = view(iterate(t));
            gv.val = w.gbuf[cur];
            run_adjoint_step(view(iterate(t - 1)), gv, log[t - 1].tau, log[t - 1].branch, w.gbuf[1 - cur], w.aw, s);
            cur = 1 - cur;
        }
    }
    // X~_0 = mask((lmax I - F) / (lmax - lmin)) with the same bounds as the forward run
    launch_gersch(view(F), w.rowtmp, w.lam, s);
    launch_adj_fbar(view(F), tape[0].map, w.gbuf[cur], w.lam, fbar_val, s);
    int32_t ovf[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&ovf[0], w.aw.ovf, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (every > 1) HIP_TRY(hipMemcpyAsync(&ovf[1], w.mw.ovf, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    if (ovf[0] || ovf[1]) return fail(SPAMM_ECAPACITY, "adjoint pair list exceeded %lld pairs", (long long)max_pairs);
    return SPAMM_OK;
}

// ---------------------------------------------------------------------------
// Batched purification of independent systems
// ---------------------------------------------------------------------------
size_t purify_sp2_batched_workspace_bytes(int32_t nsys, const spamm_bsm* F, const sp2_params* p,
                                          const int64_t* cap_blocks, const int64_t* max_pairs) {
    if (nsys < 1 || nsys > 4096 || !F || !p || !cap_blocks || !max_pairs) return 0;
    Carver c(nullptr);
    for (int q = 0; q < nsys; ++q) {
        if (F[q].nb < 1 || p[q].N < 1 || cap_blocks[q] < 1 || max_pairs[q] < 0) return 0;
        Sp2Ws w;
        carve_sp2(c, F[q].nb, F[q].b, p[q].N, cap_blocks[q], max_pairs[q], 0, w, p[q].precision, true);
    }
    c.take<GemmArgs>(2 * (size_t)nsys);        // descriptors, two parities
    c.take<int64_t>(2 * (size_t)(nsys + 1) * kBatchGroups);  // out_off / pair_off per group
    c.take<int32_t>(16 * kBatchGroups);                     // work counters per group
    c.take<Sp2Ctl*>(nsys);
    c.take<int32_t>(4);
    return c.off + 256;
}

}  // extern "C"

namespace {

__global__ void k_all_done(Sp2Ctl* const* __restrict__ ctls, int nsys, int32_t* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int all = 1;
    for (int q = 0; q < nsys; ++q) all &= ctls[q]->done ? 1 : 0;
    *out = all;
}

}  // namespace

extern "C" {

int purify_sp2_batched(int32_t nsys, const spamm_bsm* F, const sp2_params* p, spamm_bsm* D,
                       const int64_t* max_pairs, sp2_iter_log* log, int32_t log_stride, int32_t* nlog_out,
                       int32_t* status_out, void* ws, size_t ws_bytes, spamm_stream_t stream) {
    if (nsys < 1 || nsys > 4096) return fail(SPAMM_EINVAL, "nsys must be in 1..4096");
    if (!F || !p || !D || !max_pairs || !log || !nlog_out || !status_out) return fail(SPAMM_EINVAL, "NULL argument");
    std::vector<int64_t> caps(nsys);
    for (int q = 0; q < nsys; ++q) {
        int rc = check_sp2(&F[q], &p[q], &D[q]);
        if (rc) return fail(rc, "system %d: %s", q, std::string(g_err).c_str());
        if (p[q].keep_tape) return fail(SPAMM_EINVAL, "system %d: the batched loop keeps no tape", q);
        if (log_stride < p[q].n_max + 2) return fail(SPAMM_EINVAL, "log_stride must be at least n_max + 2");
        if (max_pairs[q] < 1 || max_pairs[q] >= ((int64_t)1 << 31))
            return fail(SPAMM_EINVAL, "system %d: max_pairs out of range", q);
        caps[q] = D[q].cap;
    }
    const size_t need = purify_sp2_batched_workspace_bytes(nsys, F, p, caps.data(), max_pairs);
    if (!ws || ws_bytes < need) return fail(SPAMM_EWORKSPACE, "batched purification needs %zu workspace bytes", need);
    hipStream_t s = (hipStream_t)stream;
    Carver c(ws);
    std::vector<Sp2Ws> W(nsys);
    for (int q = 0; q < nsys; ++q) {
        carve_sp2(c, F[q].nb, F[q].b, p[q].N, caps[q], max_pairs[q], 0, W[q], p[q].precision, true);
        // D[q] is the second ping-pong iterate: one matrix of capacity less per system
        W[q].X[1] = D[q];
        W[q].X[1].n = (int64_t)F[q].nb * F[q].b;
    }
    GemmArgs* descs_dev = c.take<GemmArgs>(2 * (size_t)nsys);
    int64_t* offs = c.take<int64_t>(2 * (size_t)(nsys + 1) * kBatchGroups);
    int32_t* counters = c.take<int32_t>(16 * kBatchGroups);
    Sp2Ctl** ctls_dev = c.take<Sp2Ctl*>(nsys);
    int32_t* all_done = c.take<int32_t>(4);
    if (c.off > ws_bytes) return fail(SPAMM_EWORKSPACE, "workspace too small");

    // groups of systems sharing one product launch: same leaf size and tier
    struct Group {
        int b;
        int low;  // tier: 0 FP64, 1 FP32, 2 split BF16
        std::vector<int> sys;
    };
    std::vector<Group> groups;
    for (int q = 0; q < nsys; ++q) {
        const int low = p[q].precision;
        int gi = -1;
        for (size_t k = 0; k < groups.size(); ++k)
            if (groups[k].b == F[q].b && groups[k].low == low) gi = (int)k;
        if (gi < 0) {
            groups.push_back({F[q].b, low, {}});
            gi = (int)groups.size() - 1;
        }
        groups[gi].sys.push_back(q);
    }
    if ((int)groups.size() > kBatchGroups) return fail(SPAMM_EINVAL, "more than %d product groups", kBatchGroups);

    // prologue of every system: X_0, its norms, the Gerschgorin bounds
    std::vector<int32_t> nf(nsys);
    std::vector<double> lam(2 * (size_t)nsys);
    for (int q = 0; q < nsys; ++q) {
        Sp2Ws& w = W[q];
        fill_i32(w.mw.ovf, 1, 0, s);
        fill_i32(w.sw.ovf, 1, 0, s);
        fill_i64(w.tstats, 4, 0, s);
        launch_traces_init(w.trace_tmp, s);
        MatView Fv = view(&F[q]);
        MatView X0 = view(&w.X[0]);
        launch_gersch(Fv, w.rowtmp, w.lam, s);
        launch_x0(Fv, w.lam, X0, w.dflag, w.dpos, w.mw.scan_tmp, w.dcount, s);
        launch_norms(F[q].b, X0.nslot, X0.cap, X0.brow, X0.val, X0.sq, X0.sqlo, X0.norm, s);
        HIP_TRY(hipMemcpyAsync(&lam[2 * q], w.lam, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&nf[q], F[q].nslot, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<Sp2Ctl*> ctl_ptrs(nsys);
    for (int q = 0; q < nsys; ++q) {
        const sp2_params* pq = &p[q];
        Sp2Ws& w = W[q];
        if (nf[q] + F[q].nb > caps[q] && caps[q] < (int64_t)F[q].nb * F[q].nb)
            return fail(SPAMM_ECAPACITY, "system %d: D->cap must be at least min(nslot(F) + nb, nb^2)", q);
        const bool have_gap = !isnan(pq->homo) && !isnan(pq->lumo);
        const double Wd = lam[2 * q + 1] - lam[2 * q];
        const double xh = have_gap ? (lam[2 * q + 1] - pq->homo) / Wd : NAN;
        const double xl = have_gap ? (lam[2 * q + 1] - pq->lumo) / Wd : NAN;
        Sp2Ctl hc;
        memset(&hc, 0, sizeof(hc));
        hc.delta = step_delta(pq, xh - xl);
        hc.eps = pq->eps;
        hc.homo = pq->homo;
        hc.lumo = pq->lumo;
        hc.delta_const = pq->delta_const;
        hc.e_tol = pq->e_tol;
        hc.n_occ = pq->n_occ;
        hc.n_max = pq->n_max;
        hc.variant = pq->variant;
        hc.N = pq->N;
        hc.xh = xh;
        hc.xl = xl;
        hc.tiered = pq->precision != 0 ? 1 : 0;
        hc.have_gap = have_gap ? 1 : 0;
        hc.tier_split = pq->tier_split;
        hc.trunc_scale = pq->variant == 0 ? 0.5 : 1.0;
        hc.status = SPAMM_OK;
        HIP_TRY(hipMemcpyAsync(w.ctl, &hc, sizeof(hc), hipMemcpyHostToDevice, s));
        if (pq->variant != 1)
            launch_truncate(view(&w.X[0]), &w.ctl->delta, 0.0, 1.0, w.trunc_tmp, caps[q], w.tstats, w.mw.ovf, nullptr,
                            s);
        ctl_ptrs[q] = w.ctl;
    }
    HIP_TRY(hipMemcpyAsync(ctls_dev, ctl_ptrs.data(), sizeof(Sp2Ctl*) * nsys, hipMemcpyHostToDevice, s));

    // product descriptors: parity q reads X[q] and writes X[1 - q]; one
    // contiguous run of descriptors per group
    std::vector<GemmArgs> hd(2 * (size_t)nsys);
    std::vector<int> gstart(groups.size());
    {
        int pos = 0;
        for (size_t k = 0; k < groups.size(); ++k) {
            gstart[k] = pos;
            pos += (int)groups[k].sys.size();
        }
        for (int par = 0; par < 2; ++par)
            for (size_t k = 0; k < groups.size(); ++k)
                for (size_t t = 0; t < groups[k].sys.size(); ++t) {
                    const int q = groups[k].sys[t];
                    Sp2Ws& w = W[q];
                    const int low = p[q].precision;
                    GemmArgs g;
                    g.b = F[q].b;
                    g.nb = F[q].nb;
                    g.oi = w.mw.oi;
                    g.oj = w.mw.oj;
                    g.optr = w.mw.optr;
                    g.pairs = w.mw.pairs;
                    g.nout = &w.mw.sc[1];
                    g.npairs = &w.mw.sc[0];
                    g.valA = w.X[par].val;
                    g.valB = w.X[par].val;
                    g.btrans = 1;
                    g.sym = 1;
                    g.map_out = w.X[1 - par].map;
                    g.val_out = w.X[1 - par].val;
                    g.mapX = w.X[par].map;
                    g.valX = w.X[par].val;
                    g.branch = &w.ctl->branch;
                    g.counters = w.mw.counters;
                    g.ovf = w.mw.ovf;
                    g.done = &w.ctl->done;
                    g.valA32 = low == 1 ? w.x32 : nullptr;
                    g.valB32 = low == 1 ? w.x32 : nullptr;
                    g.valA16 = low == 2 ? reinterpret_cast<const uint16_t*>(w.x32) : nullptr;
                    g.valB16 = low == 2 ? reinterpret_cast<const uint16_t*>(w.x32) : nullptr;
                    g.expA = low == 2 ? w.xexp : nullptr;
                    g.expB = low == 2 ? w.xexp : nullptr;
                    g.olow = low ? w.mw.olow : nullptr;
                    // block norms of the new iterate in the epilogue; the
                    // recheck count is reset in each step before the product
                    g.sq_out = w.X[1 - par].sq;
                    g.sqlo_out = w.X[1 - par].sqlo;
                    g.nrm_out = w.X[1 - par].norm;
                    g.recheck = w.recheck;
                    g.nrecheck = &w.mw.counters[8];
                    hd[(size_t)par * nsys + gstart[k] + t] = g;
                }
    }
    HIP_TRY(hipMemcpyAsync(descs_dev, hd.data(), sizeof(GemmArgs) * hd.size(), hipMemcpyHostToDevice, s));
    (void)num_cus();

    GraphGuard gg;
    HIP_TRY(hipEventCreate(&gg.e));
    HIP_TRY(capture_stream(&gg.cs));
    HIP_TRY(hipEventRecord(gg.e, s));
    HIP_TRY(hipStreamWaitEvent(gg.cs, gg.e, 0));
    HIP_TRY(hipStreamBeginCapture(gg.cs, hipStreamCaptureModeThreadLocal));
    for (int par = 0; par < 2; ++par) {
        // decisions of every system from the traces of its current iterate
        for (int q = 0; q < nsys; ++q) {
            Sp2Ws& w = W[q];
            MatView xv = view(&w.X[par]);
            launch_traces(xv.nslot, xv.cap, F[q].b, F[q].n, xv.brow, xv.bcol, xv.val, xv.sq, xv.sqlo, w.trace_tmp,
                          w.trace_out, &w.ctl->done, gg.cs, control_tail(w));
        }
        // sweeps, kept pairs and output patterns, system by system
        for (int q = 0; q < nsys; ++q) {
            Sp2Ws& w = W[q];
            const sp2_params* pq = &p[q];
            const bool tiered = pq->precision != 0;
            const int32_t* done = &w.ctl->done;
            MatView xv = view(&w.X[par]);
            MatView nv = view(&w.X[1 - par]);
            const SymOcc occ = build_sym_occ(xv, w.mw.bitsA, w.mw.nw, w.sw.tA, w.sw.T, w.sw.l0, done, gg.cs, &w.sw);
            if (pq->variant != 2 && pq->bound_kind != 0)
                run_sweep_leaf(xv, xv, 1, pq->tau, pq->N, &w.ctl->budget_skip, 0.0, pq->bound_kind, 0, nullptr, 0.0,
                               w.bound,
                               &w.ctl->idx, &w.ctl->tau, w.sw, done, gg.cs, &occ);
            else if (pq->variant != 2)
                run_sweep(xv, xv, 1, pq->tau, pq->N, &w.ctl->budget_skip, 0.0, 0, nullptr, 0.0, w.bound, &w.ctl->idx,
                          &w.ctl->tau, w.sw, done, gg.cs, &occ);
            if (tiered) {
                if (pq->bound_kind != 0)
                    run_sweep_leaf(xv, xv, 1, pq->tau, pq->N, &w.ctl->budget, 0.0, pq->bound_kind, 1, &w.ctl->tau,
                                   tier_constant(pq->precision, F[q].b), w.bound2, &w.ctl->sidx, &w.ctl->sigma, w.sw,
                                   done, gg.cs, &occ);
                else
                    run_sweep(xv, xv, 1, pq->tau, pq->N, &w.ctl->budget, 0.0, 1, &w.ctl->tau,
                              tier_constant(pq->precision, F[q].b), w.bound2, &w.ctl->sidx, &w.ctl->sigma, w.sw, done,
                              gg.cs, &occ);
                if (pq->precision == 2)
                    launch_to_bf16x2(F[q].b, xv.nslot, xv.cap, xv.brow, xv.val, reinterpret_cast<uint16_t*>(w.x32),
                                     w.xexp, done, gg.cs);
                else
                    launch_to_f32(F[q].b, xv.nslot, xv.cap, xv.brow, xv.val, w.x32, 1, done, gg.cs);
            }
            run_pairs(xv, xv, 1, 1, &w.ctl->tau, tiered ? &w.ctl->sigma : nullptr, nv, w.fromc, w.mw, xv.map,
                      &w.ctl->branch, done, gg.cs, &occ, pq->precision == 1 ? kFp32TierNormMin : 0.0);
            fill_i32(&w.mw.counters[8], 1, 0, gg.cs);  // recheck count of the epilogue norms
        }
        // one persistent product launch per group over all its systems
        for (size_t k = 0; k < groups.size(); ++k) {
            const size_t ng = groups[k].sys.size();
            int64_t* out_off = offs + (size_t)k * 2 * (nsys + 1);
            int64_t* pair_off = out_off + (nsys + 1);
            launch_gemm_batch(groups[k].b, groups[k].low, descs_dev + (size_t)par * nsys + gstart[k], (int)ng, out_off,
                              pair_off, counters + 16 * k, num_cus(), gg.cs);
        }
        // pass-through blocks, norms and truncation of every system
        for (int q = 0; q < nsys; ++q) {
            Sp2Ws& w = W[q];
            const sp2_params* pq = &p[q];
            const int32_t* done = &w.ctl->done;
            MatView xv = view(&w.X[par]);
            MatView nv = view(&w.X[1 - par]);
            NormOut no;
            no.sq = nv.sq;
            no.sqlo = nv.sqlo;
            no.nrm = nv.norm;
            no.recheck = w.recheck;
            no.nrecheck = &w.mw.counters[8];
            launch_rest(F[q].b, nv.nslot, nv.cap, nv.brow, nv.bcol, w.fromc, F[q].nb, xv.map, xv.val, nv.val,
                        &w.ctl->branch, done, gg.cs, no);
            launch_norms_listed(F[q].b, w.recheck, &w.mw.counters[8], nv.cap, nv.brow, nv.val, nv.sq, nv.sqlo,
                                nv.norm, gg.cs, done);
            if (pq->variant != 1)
                launch_truncate(nv, &w.ctl->delta, 0.0, pq->variant == 0 ? 0.5 : 1.0, w.trunc_tmp, caps[q], w.tstats,
                                w.mw.ovf, done, gg.cs);
        }
    }
    hipLaunchKernelGGL(k_all_done, dim3(1), dim3(64), 0, gg.cs, ctls_dev, nsys, all_done);
    hipError_t ec = hipStreamEndCapture(gg.cs, &gg.g);
    if (ec != hipSuccess) return fail(SPAMM_EHIP, "graph capture: %s", hipGetErrorString(ec));
    HIP_TRY(hipGraphInstantiate(&gg.ge, gg.g, nullptr, nullptr, 0));
    int n_max = 1, poll = 1;
    for (int q = 0; q < nsys; ++q) {
        n_max = std::max(n_max, p[q].n_max);
        poll = std::max(poll, p[q].graph_steps);
    }
    const int per_poll = std::max(1, (poll + 1) / 2);
    const int max_replays = n_max / 2 + 2;
    int32_t done = 0;
    for (int r = 0; r < max_replays && !done;) {
        for (int k = 0; k < per_poll && r < max_replays; ++k, ++r) HIP_TRY(hipGraphLaunch(gg.ge, gg.cs));
        HIP_TRY(hipMemcpyAsync(&done, all_done, sizeof(done), hipMemcpyDeviceToHost, gg.cs));
        HIP_TRY(hipStreamSynchronize(gg.cs));
    }
    if (!done) return fail(SPAMM_EHIP, "batched loop did not reach its stop");
    int worst = SPAMM_OK;
    for (int q = 0; q < nsys; ++q) {
        Sp2Ws& w = W[q];
        Sp2Ctl cs;
        HIP_TRY(hipMemcpy(&cs, w.ctl, sizeof(cs), hipMemcpyDeviceToHost));
        const int nl = cs.nlog;
        if (nl > 0) HIP_TRY(hipMemcpy(log + (size_t)q * log_stride, w.dlog, sizeof(sp2_iter_log) * nl,
                                      hipMemcpyDeviceToHost));
        nlog_out[q] = nl;
        status_out[q] = tau_fallback_status(cs.status, log + (size_t)q * log_stride, nl, p[q].variant, p[q].N);
        cs.status = status_out[q];
        if (cs.status < 0) {
            worst = cs.status;
            continue;
        }
        if (cs.status > 0 && worst == SPAMM_OK) worst = cs.status;
        // the final iterate lives in X[0] (workspace) or X[1] (= D[q] itself)
        if (((nl - 1) & 1) == 0) {
            int rc = copy_mat(D[q], w.X[0], caps[q], s);
            if (rc) return rc;
        }
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (worst < 0) return fail(worst, "a system of the batch failed (see status_out)");
    return worst;
}

// ---------------------------------------------------------------------------
// Re-blocking, product schedule, leaf-size autotuner
// ---------------------------------------------------------------------------
static int reblock_grid_p(int nb) {
    int P = 1;
    while (P < nb) P <<= 1;
    return P;
}

size_t spamm_reblock_workspace_bytes(int32_t nb_to) {
    if (nb_to < 1) return 0;
    const int64_t PP = (int64_t)reblock_grid_p(nb_to) * reblock_grid_p(nb_to);
    Carver c(nullptr);
    c.take<int32_t>(PP);
    c.take<int32_t>(PP);
    c.take<int64_t>(2);
    c.take<int32_t>(2);
    c.take<char>(scan_temp_bytes(PP));
    return c.off + 256;
}

int spamm_reblock(const spamm_bsm* X, spamm_bsm* Y, void* ws, size_t ws_bytes, spamm_stream_t stream) {
    int rc = check_bsm(X, "X", false);
    if (!rc) rc = check_bsm(Y, "Y", true);
    if (rc) return rc;
    if (X->n != Y->n) return fail(SPAMM_EINVAL, "X and Y must have the same n");
    const size_t need = spamm_reblock_workspace_bytes(Y->nb);
    if (!ws || ws_bytes < need) return fail(SPAMM_EWORKSPACE, "reblock needs %zu workspace bytes", need);
    hipStream_t s = (hipStream_t)stream;
    const int64_t PP = (int64_t)reblock_grid_p(Y->nb) * reblock_grid_p(Y->nb);
    Carver c(ws);
    int32_t* flag = c.take<int32_t>(PP);
    int32_t* pos = c.take<int32_t>(PP);
    int64_t* total = c.take<int64_t>(2);
    int32_t* ovf = c.take<int32_t>(2);
    void* tmp = c.take<char>(scan_temp_bytes(PP));
    fill_i32(ovf, 1, 0, s);
    launch_reblock(view(X), view(Y), flag, pos, total, tmp, ovf, s);
    launch_norms(Y->b, Y->nslot, Y->cap, Y->brow, Y->val, Y->sq, Y->sqlo, Y->norm, s);
    int32_t o = 0;
    int64_t t = 0;
    HIP_TRY(hipMemcpyAsync(&o, ovf, sizeof(o), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&t, total, sizeof(t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    if (o) return fail(SPAMM_ECAPACITY, "Y needs %lld slots, has %lld", (long long)t, (long long)Y->cap);
    return SPAMM_OK;
}

int spamm_set_gemm_schedule(int32_t b, int32_t workgroups_per_cu) {
    if (b != 32 && b != 64 && b != 128) return fail(SPAMM_EINVAL, "leaf size must be 32, 64 or 128");
    if (workgroups_per_cu == 0) workgroups_per_cu = b == 32 ? 4 : (b == 64 ? 3 : 2);
    if (workgroups_per_cu < 1 || workgroups_per_cu > 8) return fail(SPAMM_EINVAL, "workgroups per CU in 1..8");
    set_ring_per_cu(b, workgroups_per_cu);
    return SPAMM_OK;
}

int spamm_get_gemm_schedule(int32_t b) {
    if (b != 32 && b != 64 && b != 128) return fail(SPAMM_EINVAL, "leaf size must be 32, 64 or 128");
    return get_ring_per_cu(b);
}

int spamm_set_small_path(int32_t on) {
    if (on != 0 && on != 1) return fail(SPAMM_EINVAL, "small-system path switch must be 0 or 1");
    set_small_path(on != 0);
    return SPAMM_OK;
}

int spamm_get_small_path(void) { return small_path_enabled() ? 1 : 0; }

}  // extern "C"

namespace {

// sizes of one autotuner trial at leaf b
struct TrialSize {
    int nb;
    int64_t cap, max_pairs;
    size_t bytes;
};

TrialSize trial_size(int64_t n, int b, int N, int precision) {
    TrialSize t;
    t.nb = (int)((n + b - 1) / b);
    t.cap = (int64_t)t.nb * t.nb;
    t.max_pairs = t.cap * (t.nb + 1) / 2;
    Carver c(nullptr);
    spamm_bsm m;
    carve_mat(c, n, b, t.cap, m);  // F at leaf b
    carve_mat(c, n, b, t.cap, m);  // D at leaf b
    c.take<char>(spamm_reblock_workspace_bytes(t.nb));
    c.take<char>(purify_sp2_workspace_bytes(t.nb, b, N, t.cap, 0, 0, precision) + 8 * (size_t)t.max_pairs + 1024);
    t.bytes = c.off + 256;
    return t;
}

}  // namespace

extern "C" {

size_t purify_sp2_autotune_workspace_bytes(int64_t n, int32_t N, int32_t precision) {
    if (n < 1 || N < 1) return 0;
    size_t m = 0;
    for (int b : {32, 64, 128}) {
        if (precision != 0 && b > 64) continue;  // the precision tiers run at leaf 32 and 64
        m = std::max(m, trial_size(n, b, N, precision).bytes);
    }
    return m;
}

int purify_sp2_autotune(const spamm_bsm* F, const sp2_params* p, int32_t trial_steps, int32_t* best_b,
                        int32_t* best_per_cu, float* ms_per_step, void* ws, size_t ws_bytes, spamm_stream_t stream) {
    int rc = check_bsm(F, "F", false);
    if (rc) return rc;
    if (!p || !best_b || !best_per_cu || !ms_per_step) return fail(SPAMM_EINVAL, "NULL argument");
    if (trial_steps < 2 || trial_steps > 1000) return fail(SPAMM_EINVAL, "trial_steps must be in 2..1000");
    const size_t need = purify_sp2_autotune_workspace_bytes(F->n, p->N, p->precision);
    if (!ws || ws_bytes < need) return fail(SPAMM_EWORKSPACE, "autotune needs %zu workspace bytes", need);
    hipStream_t s = (hipStream_t)stream;
    sp2_params pt = *p;
    pt.keep_tape = 0;
    pt.graph_steps = 0;
    std::vector<sp2_iter_log> logs(trial_steps + 2);
    // mean time of the trial steps after the first, and of their products
    auto trial = [&](int b, float* ms_step, float* ms_gemm) -> int {
        const TrialSize t = trial_size(F->n, b, p->N, p->precision);
        Carver c(ws);
        spamm_bsm Fb, Db;
        carve_mat(c, F->n, b, t.cap, Fb);
        carve_mat(c, F->n, b, t.cap, Db);
        const size_t rb = spamm_reblock_workspace_bytes(t.nb);
        void* rws = c.take<char>(rb);
        int r = spamm_reblock(F, &Fb, rws, rb, stream);
        if (r) return r;
        const size_t pb = purify_sp2_workspace_bytes(t.nb, b, p->N, t.cap, 0, 0, p->precision) +
                          8 * (size_t)t.max_pairs + 1024;
        void* pws = c.take<char>(pb);
        int32_t nl = 0;
        r = purify_run(&Fb, &pt, &Db, logs.data(), &nl, pws, pb, stream, trial_steps);
        if (r < 0) return r;
        double tot = 0.0, gem = 0.0;
        int cnt = 0;
        for (int k = 1; k < nl; ++k) {
            if (logs[k].branch < 0) continue;
            tot += logs[k].ms_total;
            gem += logs[k].ms_gemm;
            ++cnt;
        }
        *ms_step = cnt ? (float)(tot / cnt) : -1.0f;
        *ms_gemm = cnt ? (float)(gem / cnt) : -1.0f;
        return SPAMM_OK;
    };
    int bb = 0;
    float best = 0.0f;
    const int leaves[3] = {32, 64, 128};
    for (int q = 0; q < 3; ++q) {
        ms_per_step[q] = -1.0f;
        if (p->precision != 0 && leaves[q] > 64) continue;  // tiers: leaf 32 and 64 only
        float st = 0.0f, gm = 0.0f;
        rc = trial(leaves[q], &st, &gm);
        if (rc) return rc;
        ms_per_step[q] = st;
        if (st > 0.0f && (bb == 0 || st < best)) {
            bb = leaves[q];
            best = st;
        }
    }
    if (bb == 0) return fail(SPAMM_EINVAL, "the trials took no step (the input converged at once)");
    // schedule of the chosen leaf: workgroups per CU of the product kernel
    const int def = get_ring_per_cu(bb);
    int best_pc = def;
    float best_g = 0.0f;
    for (int pc = 1; pc <= def; ++pc) {
        set_ring_per_cu(bb, pc);
        float st = 0.0f, gm = 0.0f;
        rc = trial(bb, &st, &gm);
        if (rc) {
            set_ring_per_cu(bb, def);
            return rc;
        }
        if (gm > 0.0f && (best_g == 0.0f || gm < best_g)) {
            best_g = gm;
            best_pc = pc;
        }
    }
    set_ring_per_cu(bb, best_pc);
    *best_b = bb;
    *best_per_cu = best_pc;
    (void)s;
    return SPAMM_OK;
}

}  // extern "C"
