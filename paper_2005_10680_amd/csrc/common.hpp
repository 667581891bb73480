// Shared device helpers and launcher declarations of the gfx950 SpAMM
// library.  Everything in here is internal; the C ABI lives in api.hip and
// include/spamm.h.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define SPAMM_DEV __device__ __forceinline__
#define SPAMM_HD __host__ __device__ __forceinline__

namespace spamm {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Morton codes.  2D: (r, c) -> bits r_k at 2k+1, c_k at 2k, so the quadrant
// order is (0,0), (0,1), (1,0), (1,1) at every level of the quadtree.
// 3D (product recursion): (i, k, j) -> i_b at 3b+2, k_b at 3b+1, j_b at 3b,
// so the low 3 bits of a node key are the octant (a, kappa, c) inside its
// parent.
// ---------------------------------------------------------------------------
SPAMM_HD uint32_t spread2(uint32_t x) {
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}
SPAMM_HD uint32_t compact2(uint32_t x) {
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return x;
}
SPAMM_HD uint32_t morton2(uint32_t r, uint32_t c) { return (spread2(r) << 1) | spread2(c); }
SPAMM_HD void demorton2(uint32_t z, uint32_t& r, uint32_t& c) {
    r = compact2(z >> 1);
    c = compact2(z);
}
SPAMM_HD uint32_t spread3(uint32_t x) {
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}
SPAMM_HD uint32_t compact3(uint32_t x) {
    x &= 0x09249249u;
    x = (x | (x >> 2)) & 0x030C30C3u;
    x = (x | (x >> 4)) & 0x0300F00Fu;
    x = (x | (x >> 8)) & 0x030000FFu;
    x = (x | (x >> 16)) & 0x000003FFu;
    return x;
}
SPAMM_HD uint32_t morton3(uint32_t i, uint32_t k, uint32_t j) {
    return (spread3(i) << 2) | (spread3(k) << 1) | spread3(j);
}
SPAMM_HD void demorton3(uint32_t z, uint32_t& i, uint32_t& k, uint32_t& j) {
    i = compact3(z >> 2);
    k = compact3(z >> 1);
    j = compact3(z);
}

// ---------------------------------------------------------------------------
// Error-free transformations (Knuth two-sum, Dekker fast two-sum, FMA
// two-product) and double-double accumulation.  The library is compiled with
// -ffp-contract=off, so each operator below is one rounding.
// ---------------------------------------------------------------------------
struct dd {
    double hi, lo;
};
SPAMM_DEV void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
SPAMM_DEV void quick_two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    e = b - (s - a);
}
SPAMM_DEV dd dd_add(dd x, dd y) {
    double s, e;
    two_sum(x.hi, y.hi, s, e);
    e = e + (x.lo + y.lo);
    dd r;
    quick_two_sum(s, e, r.hi, r.lo);
    return r;
}
SPAMM_DEV dd dd_shfl_xor(dd x, int m) {
    dd r;
    r.hi = __shfl_xor(x.hi, m);
    r.lo = __shfl_xor(x.lo, m);
    return r;
}
SPAMM_DEV dd dd_wave_sum(dd x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x = dd_add(x, dd_shfl_xor(x, m));
    return x;
}

// dd_add that reports whether it was exact: x + y = r.hi + r.lo exactly when
// neither intermediate sum of the low parts rounded (inexact stays false).
SPAMM_DEV dd dd_add_checked(dd x, dd y, bool& inexact) {
    double s, e, t, te, u, ue;
    two_sum(x.hi, y.hi, s, e);
    two_sum(x.lo, y.lo, t, te);
    two_sum(e, t, u, ue);
    if (te != 0.0 || ue != 0.0) inexact = true;
    dd r;
    two_sum(s, u, r.hi, r.lo);
    return r;
}

// Sum of squares of a block's entries, for its exactly rounded norm: each
// square is split exactly (x*x and fma(x, x, -x*x)) and accumulated in
// double-double, in any order; the flags mark entries whose square may
// overflow (special) or lose bits below the normal range (tiny).
struct SqAcc {
    dd acc = {0.0, 0.0};
    bool special = false, tiny = false;
};
SPAMM_DEV void sq_add(SqAcc& a, double x) {
    const double ax = fabs(x);
    if (!(ax < 0x1p500)) a.special = true;          // huge, inf or NaN
    if (ax != 0.0 && ax < 0x1p-480) a.tiny = true;   // two-product may be inexact
    const double p = x * x;
    const double pe = fma(x, x, -p);
    a.acc = dd_add(a.acc, dd{p, pe});
}
// Whether acc.hi is the exactly rounded sum of squares: acc = hi + lo (the
// whole block, at most 2^14 terms) is within hi * 2^-80 of the exact sum, so
// hi is certain when hi + lo lies farther than that from the nearest
// rounding boundary (hi + ulp/2 above, hi - ulp/2 below).
SPAMM_DEV bool sq_certified(dd acc, bool special, bool tiny) {
    if (special) return false;
    const double eb = acc.hi * 0x1p-80 + (tiny ? 0x1p-1000 : 0.0);
    if (acc.lo >= 0.0) {
        const double up = nextafter(acc.hi, INFINITY) - acc.hi;
        return (up - 2.0 * acc.lo) > 2.0 * eb;
    }
    const double dn = acc.hi - nextafter(acc.hi, 0.0);
    return (dn + 2.0 * acc.lo) > 2.0 * eb;
}

// inclusive scan of one int64 per thread across a block of THREADS threads
template <int THREADS = 256>
SPAMM_DEV int64_t block_inclusive_scan(int64_t v, int64_t* sh_wave, int64_t& block_total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t o = __shfl_up(v, d);
        if (lane >= d) v += o;
    }
    if (lane == 63) sh_wave[w] = v;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < THREADS / 64; ++q) {
        int64_t t = sh_wave[q];
        if (q < w) off += t;
        tot += t;
    }
    __syncthreads();
    block_total = tot;
    return v + off;
}

// ---------------------------------------------------------------------------
// Device control block of one purification (all decisions stay on device).
// ---------------------------------------------------------------------------
struct Sp2Ctl {
    // inputs
    double eps, homo, lumo, delta_const, e_tol;
    int64_t n_occ;
    int32_t n_max, variant, N, pad0;
    // state
    int32_t i, done, branch, idx;
    int32_t overflow, pad1, pad2, pad3;
    double xh, xl, delta, budget, tau;
    double t1, t2, e;
    double e_hist[3];  // e of the last three iterates (most recent first)
    int32_t n_e;       // number of valid e_hist entries
    int32_t pad4;
    // trace partials (double-double), filled by the traces kernels
    double tr_hi[2], tr_lo[2];
    // integer results of the current step
    int64_t npairs, nout, nslot_hat, ncubes, removed_units, removed_ksum;
    uint64_t trunc_thr;
    int64_t ncand;
    double trunc_Q;
    int64_t trunc_kt;
    // precision tiers: low-precision limit sigma and its candidate index
    double sigma, budget_skip;
    int32_t sidx, pad5;
    // device-driven loop: inputs of the decision rules and the run's status
    double tier_split, trunc_scale;
    int32_t tiered, have_gap, nlog, status;
};

// ---------------------------------------------------------------------------
// Decision rules of the purification loop, shared by the host loop and the
// device control kernel so both take identical decisions (double precision,
// one rounding per operation, no contraction).
// ---------------------------------------------------------------------------
// delta_i = eps * g / (2 sqrt(2) (n_max + 1)) from the mapped gap g, or the
// given constant.  Each step perturbs the iterate by < delta_i (Frobenius),
// which moves the occupied projector by at most sqrt(2) delta_i / g
// (Davis-Kahan, first order); over X~_0 and n_max steps that is eps / 2.
SPAMM_HD double sp2_step_delta(double eps, int n_max, double delta_const, double gap) {
    if (!(delta_const != delta_const)) return delta_const;  // not NaN: explicit delta
    return eps * gap / (2.8284271247461903 * (double)(n_max + 1));
}
// SP2: x^2 (0) when its trace lands closer to n_occ, else 2x - x^2 (1)
SPAMM_HD int sp2_choose_branch(double t1, double t2, int64_t n_occ) {
    const double no = (double)n_occ;
    return fabs(t2 - no) <= fabs((2.0 * t1 - t2) - no) ? 0 : 1;
}
SPAMM_HD double sp2_map_gap(double x, int br) { return br == 0 ? x * x : 2.0 * x - x * x; }
// stop when |e_i| <= e_tol, or when two steps failed to converge
// quadratically: |e_{i-2}| <= 1/8 and |e_i| > 4 e_{i-2}^2 / (1 - 2|e_{i-2}|)^2.
// With e = sum over eigenvalues of d (1 - d), d the distance to {0, 1}, two
// SP2 steps take every d to at most 4 d^2, and e <= 1/8 keeps every d below
// 2e, so exact arithmetic stays under the bound; above it, rounding, SpAMM
// and truncation errors dominate and further steps do not converge.
// e: the last n_e values, most recent first (n_e <= 3).
SPAMM_HD bool sp2_should_stop(const double* e, int n_e, double e_tol) {
    if (n_e < 1) return false;
    if (fabs(e[0]) <= e_tol) return true;
    if (n_e >= 3) {
        const double a = fabs(e[2]);
        if (a <= 0.125) {
            const double d = 1.0 - 2.0 * a;
            if (fabs(e[0]) > 4.0 * a * a / (d * d)) return true;
        }
    }
    return false;
}
// RN(a - b) for double-doubles a = ahi + alo, b = bhi + blo
SPAMM_HD double dd_diff(double ahi, double alo, double bhi, double blo) {
    double s = ahi - bhi;
    double bb = s - ahi;
    double e = (ahi - (s - bb)) + (-bhi - bb);
    e = e + (alo - blo);
    return s + e;
}
// quantum of the truncation keys: 2^(floor(log2 RN(delta^2)) - 40)
SPAMM_HD double sp2_trunc_quantum(double delta) {
    const double T = delta * delta;
    if (!(T > 0.0) || !(T <= 1.7976931348623157e308)) return 0.0;
    int e;
    frexp(T, &e);
    int eq = e - 1 - 40;
    if (eq < -1000) eq = -1000;
    return ldexp(1.0, eq);
}

// flags in Sp2Ctl::overflow
constexpr int kOvfPairs = 1, kOvfOut = 2, kOvfSlots = 4, kOvfCubes = 8, kOvfCand = 16;

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files).  All take a hipStream_t and enqueue.
// ---------------------------------------------------------------------------
int grid_for(int64_t items, int per_block, int max_blocks);

// scans.hip
size_t scan_temp_bytes(int64_t n);
// exclusive scan of int32 in[0..n) into out (may alias), total written to
// *total_dev (int64).  n_dev (optional) caps n on device.
void scan_i32(const int32_t* in, int32_t* out, int64_t n, const int64_t* n_dev, int64_t* total_dev,
              void* temp, hipStream_t s);
void fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s);
void fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
void fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s);
void copy_i64(int64_t* dst, const int64_t* src, hipStream_t s);

}  // namespace spamm
