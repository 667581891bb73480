// Leaf-level error bounds over the skipped block pairs (alternatives to the
// recursive bound of Algorithm 3, computed for every candidate threshold):
//   sum : B_sum(tau)  = sum over all skipped triples (i,k,j) of p_ikj,
//   flat: B_flat(tau) = sqrt(sum over outputs (i,j) of (sum_{k skipped} p_ikj)^2),
// p_ikj = RN(nu(A_ik) nu(B_kj)), skipped iff p < tau.  B_flat is eq. (6)
// applied at the leaves: ||E_ij||_F <= sum_k ||A_ik||_F ||B_kj||_F for the
// skipped k of each output block, so ||E||_F <= B_flat <= B_tree (Algorithm
// 3's bound) <= B_sum.
//
// Rounding: per output the skipped products are summed in ascending k, one
// rounding per addition (s_ij); the sum over outputs is exact and rounded
// once: B_sum = RN(sum s_ij), B_flat = sqrt_RN(RN(sum RN(s_ij^2))).  So the
// result does not depend on how the outputs are distributed over waves.
//
// One wave per output block.  The wave first gathers the output's present
// products p_ikj in ascending k into its LDS row (64 inner indices at a
// time: each lane tests one k, the lanes' loads are independent, and a
// ballot compacts the present ones), then lane m (and m + 64, ...) adds
// the p below its own threshold tau_m along that row.  The per-output terms
// go into double-double partial sums per wave; a second kernel adds the
// partials and keeps the high part when the double-double value lies
// farther from a rounding boundary than its error bound (non-negative
// terms: below 2^-80 of the sum).  A candidate whose sum misses that
// certificate is summed again exactly: its terms are added into a
// fixed-point accumulator (32-bit payloads in 64-bit words, units 2^-1074)
// with atomics, then rounded once.
#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

// fixed-point accumulator of one candidate: kLeafLimbs 64-bit words, word q
// holding a sum of 32-bit payloads of weight 2^(32q - 1074); the last word
// counts non-finite terms
constexpr int kLeafLimbs = 68;

struct LeafScratch {
    double* part;     // [waves][N][2] double-double partial sums
    int32_t* pflag;   // [waves] 1: a non-finite or huge term, 2: a tiny term
    int32_t* exflag;  // [N] 1: summed exactly
    int32_t* excount; // [1]
    unsigned long long* limbs;  // [N][kLeafLimbs]
};

static LeafScratch carve_leaf(void* scratch, int nb, int N) {
    LeafScratch t;
    char* p = (char*)scratch;
    const int64_t nw = bound_part_waves(nb);
    t.part = (double*)p;
    p += ((size_t)nw * N * 2 * 8 + 255) / 256 * 256;
    t.pflag = (int32_t*)p;
    p += ((size_t)nw * 4 + 255) / 256 * 256;
    t.exflag = (int32_t*)p;
    p += ((size_t)N * 4 + 255) / 256 * 256;
    t.excount = (int32_t*)p;
    p += 256;
    t.limbs = (unsigned long long*)p;
    return t;
}

size_t bound_leaf_scratch_bytes(int nb, int N) {
    const int64_t nw = bound_part_waves(nb);
    return ((size_t)nw * N * 2 * 8 + 255) / 256 * 256 + ((size_t)nw * 4 + 255) / 256 * 256 +
           ((size_t)N * 4 + 255) / 256 * 256 + 256 + (size_t)N * kLeafLimbs * 8;
}

// Gather the present products of output (i, j) into the wave's LDS row in
// ascending k; returns their count.
SPAMM_DEV int gather_row(int i, int j, int nb, int nw, const uint32_t* __restrict__ bitsA,
                         const uint32_t* __restrict__ bitsB, const int32_t* __restrict__ mapA,
                         const double* __restrict__ normA, const int32_t* __restrict__ mapB,
                         const double* __restrict__ normB, int btrans, double* row) {
    const int lane = threadIdx.x & 63;
    int cnt = 0;
    for (int base = 0; base < nb; base += 64) {
        const int k = base + lane;
        bool pres = false;
        double p = 0.0;
        if (k < nb) {
            const uint32_t word = bitsA[(size_t)i * nw + (k >> 5)] & bitsB[(size_t)j * nw + (k >> 5)];
            if ((word >> (k & 31)) & 1u) {
                const int sa = mapA[(size_t)i * nb + k];
                const int sb = btrans ? mapB[(size_t)j * nb + k] : mapB[(size_t)k * nb + j];
                if (sa >= 0 && sb >= 0) {
                    p = normA[sa] * normB[sb];
                    pres = true;
                }
            }
        }
        const uint64_t bal = __ballot(pres);
        if (pres) row[cnt + __popcll(bal & ((1ull << lane) - 1ull))] = p;
        cnt += __popcll(bal);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return cnt;
}

// The per-output terms of the R candidates this lane serves (lane + 64 r):
// s = k-ascending sum of the leaf values, term = RN(s^2) (flat) or s.
template <int R>
SPAMM_DEV void row_terms(const double* row, int cnt, const double (&tm)[R], int mode, double t0, double c_low,
                         int flat, double (&term)[R]) {
    double s[R];
#pragma unroll
    for (int r = 0; r < R; ++r) s[r] = 0.0;
    if (mode == 0) {
        for (int q = 0; q < cnt; ++q) {
            const double p = row[q];
#pragma unroll
            for (int r = 0; r < R; ++r) s[r] = (p < tm[r]) ? s[r] + p : s[r];
        }
    } else {
        // tier mode: p below tau0 is skipped (p), from tau0 up to the
        // candidate sigma it runs in the low tier (c_low p)
        for (int q = 0; q < cnt; ++q) {
            const double p = row[q];
            const double cp = c_low * p;
#pragma unroll
            for (int r = 0; r < R; ++r) s[r] = (p < t0) ? s[r] + p : ((p < tm[r]) ? s[r] + cp : s[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) term[r] = flat ? s[r] * s[r] : s[r];
}

template <int R>
__global__ __launch_bounds__(256) void k_bound_part(int nb, int nw, const uint32_t* __restrict__ bitsA,
                                                   const uint32_t* __restrict__ bitsB,
                                                   const int32_t* __restrict__ mapA, const double* __restrict__ normA,
                                                   const int32_t* __restrict__ mapB, const double* __restrict__ normB,
                                                   int btrans, const double* __restrict__ tau, int N, int flat,
                                                   int mode, const double* __restrict__ tau0_p, double c_low,
                                                   LeafScratch ls, const int32_t* __restrict__ done) {
    extern __shared__ double prow[];  // [4][nb]
    if (done && *done) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) *ls.excount = 0;
    const double t0 = (mode == 1 && tau0_p) ? *tau0_p : 0.0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double* row = prow + (size_t)w * nb;
    double tm[R];
    dd acc[R];
    bool huge = false, tiny = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int m = lane + 64 * r;
        tm[r] = m < N ? tau[m] : 0.0;
        acc[r] = dd{0.0, 0.0};
    }
    const int64_t nout = (int64_t)nb * nb;
    const int64_t wid = (int64_t)blockIdx.x * 4 + w, nwaves = (int64_t)gridDim.x * 4;
    for (int64_t z = wid; z < nout; z += nwaves) {
        const int i = (int)(z / nb), j = (int)(z % nb);
        const int cnt = gather_row(i, j, nb, nw, bitsA, bitsB, mapA, normA, mapB, normB, btrans, row);
        double term[R];
        row_terms<R>(row, cnt, tm, mode, t0, c_low, flat, term);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double t = term[r];
            if (!(t < 0x1p1000)) huge = true;           // huge, inf or NaN
            else if (t != 0.0 && t < 0x1p-900) tiny = true;  // error terms may underflow
            acc[r] = dd_add(acc[r], dd{t, 0.0});
        }
        // the row is rewritten by the next output: every lane must be done reading
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int m = lane + 64 * r;
        if (m < N) {
            ls.part[((size_t)wid * N + m) * 2] = acc[r].hi;
            ls.part[((size_t)wid * N + m) * 2 + 1] = acc[r].lo;
        }
    }
    const int fl = (__any(huge) ? 1 : 0) | (__any(tiny) ? 2 : 0);
    if (lane == 0) ls.pflag[wid] = fl;
}

// One workgroup per candidate: thread t adds partials t, t + 256, ... in
// order, a fixed-shape tree adds the 256 thread sums (double-double); the
// rounded sum is kept when certified, else the candidate is listed for the
// exact pass.  Also clears the candidate's exact accumulator.
__global__ __launch_bounds__(256) void k_bound_final(LeafScratch ls, int64_t nparts, int N, int flat,
                                                    double* __restrict__ out, const int32_t* __restrict__ done) {
    __shared__ double rh[256], rl[256];
    __shared__ int rf[256];
    if (done && *done) return;
    const int m = blockIdx.x;
    if (threadIdx.x < kLeafLimbs) ls.limbs[(size_t)m * kLeafLimbs + threadIdx.x] = 0ull;
    dd t = {0.0, 0.0};
    int fl = 0;
    for (int64_t q = threadIdx.x; q < nparts; q += 256) {
        t = dd_add(t, dd{ls.part[((size_t)q * N + m) * 2], ls.part[((size_t)q * N + m) * 2 + 1]});
        fl |= ls.pflag[q];
    }
    rh[threadIdx.x] = t.hi;
    rl[threadIdx.x] = t.lo;
    rf[threadIdx.x] = fl;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const dd u = dd_add(dd{rh[threadIdx.x], rl[threadIdx.x]}, dd{rh[threadIdx.x + h], rl[threadIdx.x + h]});
            rh[threadIdx.x] = u.hi;
            rl[threadIdx.x] = u.lo;
            rf[threadIdx.x] |= rf[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const dd S = {rh[0], rl[0]};
        if (sq_certified(S, (rf[0] & 1) != 0, (rf[0] & 2) != 0)) {
            out[m] = flat ? sqrt(S.hi) : S.hi;
            ls.exflag[m] = 0;
        } else {
            ls.exflag[m] = 1;
            atomicAdd(ls.excount, 1);
        }
    }
}

// add the non-negative double t exactly into the accumulator L
SPAMM_DEV void limbs_add_term(unsigned long long* L, double t) {
    if (t == 0.0) return;
    if (!isfinite(t)) {
        atomicAdd(&L[kLeafLimbs - 1], 1ull);
        return;
    }
    const uint64_t bits = (uint64_t)__double_as_longlong(t);
    const int ex = (int)((bits >> 52) & 0x7ff);
    uint64_t mnt = bits & ((1ull << 52) - 1);
    int e;
    if (ex == 0) {
        e = -1074;
    } else {
        mnt |= 1ull << 52;
        e = ex - 1075;
    }
    const int pos = e + 1074, q = pos >> 5, sh = pos & 31;
    // mnt << sh spans at most 85 bits: three 32-bit payloads
    const unsigned __int128 v = (unsigned __int128)mnt << sh;
    atomicAdd(&L[q], (unsigned long long)(uint32_t)v);
    atomicAdd(&L[q + 1], (unsigned long long)(uint32_t)(v >> 32));
    atomicAdd(&L[q + 2], (unsigned long long)(uint32_t)(v >> 64));
}

// The listed candidates again, every term added exactly (one wave per
// output, as k_bound_part).  Returns at once when none is listed.
template <int R>
__global__ __launch_bounds__(256) void k_bound_exact(int nb, int nw, const uint32_t* __restrict__ bitsA,
                                                    const uint32_t* __restrict__ bitsB,
                                                    const int32_t* __restrict__ mapA, const double* __restrict__ normA,
                                                    const int32_t* __restrict__ mapB, const double* __restrict__ normB,
                                                    int btrans, const double* __restrict__ tau, int N, int flat,
                                                    int mode, const double* __restrict__ tau0_p, double c_low,
                                                    LeafScratch ls, const int32_t* __restrict__ done) {
    extern __shared__ double prow[];  // [4][nb]
    if (done && *done) return;
    if (*ls.excount == 0) return;
    const double t0 = (mode == 1 && tau0_p) ? *tau0_p : 0.0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double* row = prow + (size_t)w * nb;
    double tm[R];
    bool want[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int m = lane + 64 * r;
        tm[r] = m < N ? tau[m] : 0.0;
        want[r] = m < N && ls.exflag[m] != 0;
    }
    const int64_t nout = (int64_t)nb * nb;
    const int64_t wid = (int64_t)blockIdx.x * 4 + w, nwaves = (int64_t)gridDim.x * 4;
    for (int64_t z = wid; z < nout; z += nwaves) {
        const int i = (int)(z / nb), j = (int)(z % nb);
        const int cnt = gather_row(i, j, nb, nw, bitsA, bitsB, mapA, normA, mapB, normB, btrans, row);
        double term[R];
        row_terms<R>(row, cnt, tm, mode, t0, c_low, flat, term);
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (want[r]) limbs_add_term(ls.limbs + (size_t)(lane + 64 * r) * kLeafLimbs, term[r]);
        __builtin_amdgcn_wave_barrier();
    }
}

// Round the listed candidates' exact sums once (to nearest, ties to even).
__global__ void k_bound_exact_final(LeafScratch ls, int N, int flat, double* __restrict__ out,
                                    const int32_t* __restrict__ done) {
    if (done && *done) return;
    if (*ls.excount == 0) return;
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < N; m += gridDim.x * blockDim.x) {
        if (!ls.exflag[m]) continue;
        const unsigned long long* L = ls.limbs + (size_t)m * kLeafLimbs;
        if (L[kLeafLimbs - 1]) {
            out[m] = INFINITY;  // a non-finite term (the sum of non-negative terms)
            continue;
        }
        // normalise to 32-bit limbs
        uint32_t w[kLeafLimbs];
        unsigned long long carry = 0;
        for (int q = 0; q < kLeafLimbs - 1; ++q) {
            const unsigned long long v = L[q] + carry;
            w[q] = (uint32_t)v;
            carry = v >> 32;
        }
        w[kLeafLimbs - 1] = (uint32_t)carry;
        int top = -1;
        for (int q = kLeafLimbs - 1; q >= 0 && top < 0; --q)
            if (w[q]) top = q * 32 + 31 - __clz(w[q]);
        double v = 0.0;
        if (top >= 0) {
            // value = W * 2^-1074; keep 53 bits from the top (fewer below 2^-1022)
            int lsb = top - 52;
            if (lsb < 0) lsb = 0;
            uint64_t M = 0;
            for (int i = top; i >= lsb; --i) M = (M << 1) | ((w[i >> 5] >> (i & 31)) & 1u);
            int rb = lsb >= 1 ? (int)((w[(lsb - 1) >> 5] >> ((lsb - 1) & 31)) & 1u) : 0;
            int sticky = 0;
            for (int i = lsb - 2; i >= 0 && !sticky; --i) sticky = (int)((w[i >> 5] >> (i & 31)) & 1u);
            if (rb && (sticky || (M & 1u))) M += 1;
            v = ldexp((double)M, lsb - 1074);  // M <= 2^53: exact, or infinity on overflow
        }
        out[m] = flat ? sqrt(v) : v;
    }
}

// the LDS rows limit the leaf-level bounds to nb <= kBoundMaxNb (64 KB per workgroup)
int64_t bound_part_waves(int nb) {
    const int64_t nout = (int64_t)nb * nb;
    int64_t blocks = (nout + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    return blocks * 4;
}

void launch_bound_leaf(int nb, int nw, const uint32_t* bitsA, const uint32_t* bitsB, const int32_t* mapA,
                       const double* normA, const int32_t* mapB, const double* normB, int btrans, const double* tau,
                       int N, int flat, int mode, const double* tau0, double c_low, void* scratch, double* out,
                       const int32_t* done, hipStream_t s) {
    const LeafScratch ls = carve_leaf(scratch, nb, N);
    const int64_t nw_waves = bound_part_waves(nb);
    const int grid = (int)(nw_waves / 4);
    const size_t lds = sizeof(double) * 4 * (size_t)nb;  // one row of nb products per wave
#define SPAMM_BP(K_, R_)                                                                                        \
    hipLaunchKernelGGL((K_<R_>), dim3(grid), dim3(256), lds, s, nb, nw, bitsA, bitsB, mapA, normA, mapB, normB, \
                       btrans, tau, N, flat, mode, tau0, c_low, ls, done)
#define SPAMM_BPR(K_)                      \
    if (N <= 64) SPAMM_BP(K_, 1);          \
    else if (N <= 128) SPAMM_BP(K_, 2);    \
    else if (N <= 256) SPAMM_BP(K_, 4);    \
    else if (N <= 512) SPAMM_BP(K_, 8);    \
    else SPAMM_BP(K_, 16);
    SPAMM_BPR(k_bound_part)
    hipLaunchKernelGGL(k_bound_final, dim3(N), dim3(256), 0, s, ls, nw_waves, N, flat, out, done);
    SPAMM_BPR(k_bound_exact)
#undef SPAMM_BPR
#undef SPAMM_BP
    hipLaunchKernelGGL(k_bound_exact_final, dim3(grid_for(N, 256, 4)), dim3(256), 0, s, ls, N, flat, out, done);
}

}  // namespace spamm
