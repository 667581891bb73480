// K1: block Frobenius norms (skip test of Algorithm 2, leaf values of
// Algorithm 3) and the traces used by the purification driver.
//
// nu(X) = sqrt_RN(RN(sum x^2)): the exact sum of squares rounded once,
// then a correctly rounded square root.  One wave per block: coalesced
// 16-byte loads, double-double accumulation of the exact squares
// (x*x and fma(x, x, -x*x)), a butterfly reduction across the wave, then a
// certificate that the double-double value rounds like the exact sum.  A
// block whose sum lies too close to a rounding boundary (or holds values
// outside [2^-480, 2^500]) is summed exactly with a 32-bit-limb long
// accumulator by one lane.
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

// Long accumulator: value * 2^2148 as an unsigned integer in 32-bit limbs.
constexpr int kLimbs = 140;  // 4480 bits > 2148 + 2048 + 106 + carries

SPAMM_DEV void limbs_add128(uint32_t* L, uint64_t lo, uint64_t hi, int shift) {
    const int q = shift >> 5, o = shift & 31;
    uint32_t v[5];
    v[0] = (uint32_t)lo;
    v[1] = (uint32_t)(lo >> 32);
    v[2] = (uint32_t)hi;
    v[3] = (uint32_t)(hi >> 32);
    v[4] = 0;
    uint32_t w[5];
    if (o == 0) {
        for (int t = 0; t < 5; ++t) w[t] = v[t];
    } else {
        w[0] = v[0] << o;
        for (int t = 1; t < 5; ++t) w[t] = (v[t] << o) | (v[t - 1] >> (32 - o));
    }
    uint64_t carry = 0;
    for (int t = 0; q + t < kLimbs; ++t) {
        uint64_t s = (uint64_t)L[q + t] + carry + (t < 5 ? w[t] : 0u);
        L[q + t] = (uint32_t)s;
        carry = s >> 32;
        if (t >= 4 && carry == 0) break;
    }
}

// decompose finite nonzero x = m * 2^e, m < 2^53 integer
SPAMM_DEV void split_double(double x, uint64_t& m, int& e) {
    uint64_t bits = (uint64_t)__double_as_longlong(x);
    int ex = (int)((bits >> 52) & 0x7ff);
    m = bits & ((1ull << 52) - 1);
    if (ex == 0) {
        e = -1074;
    } else {
        m |= 1ull << 52;
        e = ex - 1075;
    }
}

SPAMM_DEV int limbs_bit(const uint32_t* L, int i) { return (int)((L[i >> 5] >> (i & 31)) & 1u); }

// round value*2^-2148 to nearest double, ties to even
SPAMM_DEV double limbs_round(const uint32_t* L) {
    int top = -1;
    for (int t = kLimbs - 1; t >= 0; --t)
        if (L[t]) {
            top = t * 32 + 31 - __clz(L[t]);
            break;
        }
    if (top < 0) return 0.0;
    if (top - 2148 >= 1024) return INFINITY;
    int lsb = top - 52;
    if (lsb < 1074) lsb = 1074;  // 2^-1074 is the subnormal step
    uint64_t M = 0;
    for (int i = top; i >= lsb; --i) M = (M << 1) | (uint64_t)limbs_bit(L, i);
    int rb = lsb >= 1 ? limbs_bit(L, lsb - 1) : 0;
    int sticky = 0;
    for (int i = lsb - 2; i >= 0 && !sticky; --i) {
        if ((i & 31) == 31 && L[i >> 5] == 0) {
            i -= 31;
            continue;
        }
        sticky = limbs_bit(L, i);
    }
    if (rb && (sticky || (M & 1u))) M += 1;
    return ldexp((double)M, lsb - 2148);
}

SPAMM_DEV double exact_sumsq_lane(const double* v, int len, uint32_t* L) {
    bool has_nan = false, has_inf = false;
    for (int t = 0; t < kLimbs; ++t) L[t] = 0;
    for (int t = 0; t < len; ++t) {
        double x = v[t];
        if (isnan(x)) { has_nan = true; continue; }
        if (isinf(x)) { has_inf = true; continue; }
        if (x == 0.0) continue;
        uint64_t m;
        int e;
        split_double(x, m, e);
        uint64_t lo = m * m, hi = __umul64hi(m, m);
        limbs_add128(L, lo, hi, 2 * e + 2148);
    }
    if (has_nan) return NAN;
    if (has_inf) return INFINITY;
    return limbs_round(L);
}

// Gerschgorin radii that the double-double row sums could not certify
// (lo[g] is NaN; hi[g] holds the centre): one thread per such row sums
// |f_gc| over c != g exactly in a long accumulator and rounds once.
__global__ __launch_bounds__(64) void k_gersch_exact(MatView F, double* __restrict__ lo, double* __restrict__ hi) {
    __shared__ uint32_t Ls[64][kLimbs];
    const int64_t n = F.n;
    const int b = F.b, nb = F.nb;
    for (int64_t g0 = (int64_t)blockIdx.x * 64; g0 < n; g0 += (int64_t)gridDim.x * 64) {
        const int64_t g = g0 + threadIdx.x;
        if (g >= n || !isnan(lo[g])) continue;
        uint32_t* L = Ls[threadIdx.x];
        for (int t = 0; t < kLimbs; ++t) L[t] = 0;
        bool has_nan = false, has_inf = false;
        const int I = (int)(g / b), r = (int)(g % b);
        for (int J = 0; J < nb; ++J) {
            const int sl = F.map[(size_t)I * nb + J];
            if (sl < 0) continue;
            const double* v = F.val + (size_t)sl * b * b;
            for (int c = 0; c < b; ++c) {
                const int64_t gj = (int64_t)J * b + c;
                if (gj >= n) break;
                if (gj == g) continue;
                const double x = fabs(v[(size_t)c * b + r]);
                if (isnan(x)) { has_nan = true; continue; }
                if (isinf(x)) { has_inf = true; continue; }
                if (x == 0.0) continue;
                uint64_t m;
                int e;
                split_double(x, m, e);
                limbs_add128(L, m, 0ull, e + 2148);
            }
        }
        const double R = has_nan ? NAN : (has_inf ? INFINITY : limbs_round(L));
        const double c0 = hi[g];
        lo[g] = c0 - R;
        hi[g] = c0 + R;
    }
}

void launch_gersch_exact(const MatView& F, double* lo, double* hi, hipStream_t s) {
    hipLaunchKernelGGL(k_gersch_exact, dim3(grid_for(F.n, 64, 1024)), dim3(64), 0, s, F, lo, hi);
}

// Exactly rounded sum of squares of slot s (one wave): double-double
// accumulation, certified; else (typically an exact tie, as with entries of
// few significant bits) the same sum again with every addition checked for
// rounding: when none rounded, the sum is exact and its leading part is the
// rounded result; else lane 0 computes it exactly.
template <int B>
SPAMM_DEV void norm_slot(int64_t s, const double* __restrict__ val, double* __restrict__ sq,
                         double* __restrict__ sqlo, double* __restrict__ nrm, uint32_t* slow) {
    const int lane = threadIdx.x & 63;
    const double2* v = reinterpret_cast<const double2*>(val + (size_t)s * B * B);
    SqAcc a;
#pragma unroll 4
    for (int it = 0; it < B * B / 128; ++it) {
        const double2 x2 = v[it * 64 + lane];
        sq_add(a, x2.x);
        sq_add(a, x2.y);
    }
    const dd acc = dd_wave_sum(a.acc);
    const bool special = __any(a.special), tiny = __any(a.tiny);
    bool ok = sq_certified(acc, special, tiny);
    double sres = acc.hi, slo = acc.lo;
    if (!ok && !special && !tiny) {
        // squares are split exactly (no entry is tiny), so only additions can round
        dd t = {0.0, 0.0};
        bool inexact = false;
        for (int it = 0; it < B * B / 128; ++it) {
            const double2 x2 = v[it * 64 + lane];
            const double xs[2] = {x2.x, x2.y};
            for (int q = 0; q < 2; ++q) {
                const double p = xs[q] * xs[q];
                t = dd_add_checked(t, dd{p, fma(xs[q], xs[q], -p)}, inexact);
            }
        }
        for (int m = 32; m >= 1; m >>= 1) t = dd_add_checked(t, dd_shfl_xor(t, m), inexact);
        if (!__any(inexact)) {
            ok = true;
            sres = t.hi;
            slo = t.lo;
        }
    }
    if (!ok) {
        if (lane == 0) {
            const double ex = exact_sumsq_lane(val + (size_t)s * B * B, B * B, slow);
            slo = (acc.hi - ex) + acc.lo;
            sres = ex;
        }
        sres = __shfl(sres, 0);
        slo = __shfl(slo, 0);
    }
    if (lane == 0) {
        sq[s] = sres;
        sqlo[s] = slo;
        nrm[s] = sqrt(sres);
    }
}

// Norms of every live slot, or (list != null) of the *nlist slots listed:
// the blocks whose norm a producing kernel could not certify.
template <int B>
__global__ __launch_bounds__(256) void k_norms(const int32_t* __restrict__ nslot_p, int64_t cap,
                                              const int32_t* __restrict__ brow, const double* __restrict__ val,
                                              double* __restrict__ sq, double* __restrict__ sqlo,
                                              double* __restrict__ nrm, const int32_t* __restrict__ done,
                                              const int32_t* __restrict__ list, const int32_t* __restrict__ nlist) {
    __shared__ uint32_t slow[4][kLimbs];
    if (done && *done) return;
    const int wv = threadIdx.x >> 6;
    int64_t nslot = list ? (int64_t)*nlist : *nslot_p;
    if (nslot > cap) nslot = cap;
    for (int64_t q = (int64_t)blockIdx.x * 4 + wv; q < nslot; q += (int64_t)gridDim.x * 4) {
        const int64_t s = list ? (int64_t)list[q] : q;
        if (brow[s] < 0) continue;  // hole (wave-uniform)
        norm_slot<B>(s, val, sq, sqlo, nrm, slow[wv]);
    }
}

void launch_norms(int b, const int32_t* nslot, int64_t cap, const int32_t* brow, const double* val, double* sq,
                  double* sqlo, double* nrm, hipStream_t s, const int32_t* done) {
    int grid = grid_for(cap, 4, 8192);
    const int32_t* nl = nullptr;
    switch (b) {
        case 32: hipLaunchKernelGGL(k_norms<32>, dim3(grid), dim3(256), 0, s, nslot, cap, brow, val, sq, sqlo, nrm, done, nl, nl); break;
        case 64: hipLaunchKernelGGL(k_norms<64>, dim3(grid), dim3(256), 0, s, nslot, cap, brow, val, sq, sqlo, nrm, done, nl, nl); break;
        case 128: hipLaunchKernelGGL(k_norms<128>, dim3(grid), dim3(256), 0, s, nslot, cap, brow, val, sq, sqlo, nrm, done, nl, nl); break;
    }
}

void launch_norms_listed(int b, const int32_t* list, const int32_t* nlist, int64_t cap, const int32_t* brow,
                         const double* val, double* sq, double* sqlo, double* nrm, hipStream_t s, const int32_t* done) {
    const int grid = 64;  // the list is empty or short
    const int32_t* ns = nullptr;
    switch (b) {
        case 32: hipLaunchKernelGGL(k_norms<32>, dim3(grid), dim3(256), 0, s, ns, cap, brow, val, sq, sqlo, nrm, done, list, nlist); break;
        case 64: hipLaunchKernelGGL(k_norms<64>, dim3(grid), dim3(256), 0, s, ns, cap, brow, val, sq, sqlo, nrm, done, list, nlist); break;
        case 128: hipLaunchKernelGGL(k_norms<128>, dim3(grid), dim3(256), 0, s, ns, cap, brow, val, sq, sqlo, nrm, done, list, nlist); break;
    }
}

// dst <- src: the slot count, the whole block map and the live slots
// (s < min(*src.nslot, cap)) with their values and norms, in one launch.
__global__ void k_copy_live(MatView src, MatView dst, int64_t cap) {
    int64_t ns = *src.nslot;
    if (ns > cap) ns = cap;
    if (ns < 0) ns = 0;
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gs = (int64_t)gridDim.x * blockDim.x;
    if (gt == 0) *dst.nslot = *src.nslot;
    const int64_t nmap = (int64_t)src.nb * src.nb;
    for (int64_t t = gt; t < nmap; t += gs) dst.map[t] = src.map[t];
    for (int64_t t = gt; t < ns; t += gs) {
        dst.brow[t] = src.brow[t];
        dst.bcol[t] = src.bcol[t];
        dst.norm[t] = src.norm[t];
        dst.sq[t] = src.sq[t];
        dst.sqlo[t] = src.sqlo[t];
    }
    const int64_t nv = ns * src.b * src.b;
    for (int64_t t = gt; t < nv; t += gs) dst.val[t] = src.val[t];
}

void launch_copy_live(const MatView& src, const MatView& dst, int64_t cap, hipStream_t s) {
    const int64_t items = std::max<int64_t>(cap * src.b * src.b, (int64_t)src.nb * src.nb);
    hipLaunchKernelGGL(k_copy_live, dim3(grid_for(items, 256, 4096)), dim3(256), 0, s, src, dst, cap);
}

}  // namespace spamm
