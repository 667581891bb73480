// K4: truncation with ||E||_F < delta (the truncation lines of Algorithms 1
// and 5) on a symmetric block matrix.
//
// Units are diagonal blocks (weight 1) and symmetric off-diagonal pairs
// (weight 2, keyed by the upper block).  With T = RN(delta^2) and the
// power-of-two quantum Q = 2^(floor(log2 T) - 40), a unit's integer key is
// k = ceil(w * sq / Q) (saturated at 2^41), and the budget is
// K_T = floor(T/Q).  Units are ordered by (k, r*nb + c) and the longest
// prefix whose key sum is < K_T is removed.  Integer keys make the prefix
// sums exact and order-independent, so the removed set is unique.  The
// bound is rigorous: a key sum of at most K_T - 1 means sum(w sq) <= T - Q
// with Q > 2^-41 T, which leaves room for the rounding of each sq (2^-53
// relative) and of T = RN(delta^2) (2^-53), so the exact removed squared
// norm stays below delta^2.
//
// Only units with k < K_T can ever be removed; they are collected first and
// the cut is found by an 8-pass radix select over the 64-bit composite key
// (k << 22 | r*nb + c) with exact per-digit key sums in LDS.
#include <math.h>

#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

constexpr int kKeyBits = 40;
constexpr uint64_t kKSat = 1ull << 41;

struct TruncQuanta {
    double Q;
    uint64_t kt;
    bool any;
};

SPAMM_DEV TruncQuanta trunc_quanta(double delta) {
    TruncQuanta q;
    double T = delta * delta;
    q.any = (T > 0.0) && isfinite(T);
    q.Q = 0.0;
    q.kt = 0;
    if (!q.any) return q;
    int e;
    frexp(T, &e);
    int eT = e - 1;
    int eq = eT - kKeyBits;
    if (eq < -1000) eq = -1000;
    q.Q = ldexp(1.0, eq);
    q.kt = (uint64_t)floor(T / q.Q);
    if (q.kt == 0) q.any = false;
    return q;
}

size_t trunc_temp_bytes(int64_t cap) {
    // cand keys + cand k + counters
    return (size_t)cap * 16 + 64;
}

struct TruncTemp {
    uint64_t* key;
    uint64_t* k;
    int64_t* ncand;  // [1]
    uint64_t* thr;   // [1]
};

static TruncTemp carve_trunc(void* temp, int64_t cap) {
    TruncTemp t;
    char* p = (char*)temp;
    t.ncand = (int64_t*)p;
    t.thr = (uint64_t*)(p + 16);
    t.key = (uint64_t*)(p + 64);
    t.k = t.key + cap;
    return t;
}

// One radix-select decision, taken by the first wave (all 64 lanes): the
// first digit b (0..255) whose bucket still fits no more, cum(b) + hs[b] >= rem
// with cum(b) = hs[0] + ... + hs[b-1], or -1 when every bucket fits.  Lane l
// owns buckets 4l .. 4l+3; a wave scan of the lane sums gives each lane its
// starting cum.  Integer sums, so the answer is the sequential scan's.
SPAMM_DEV int radix_bucket(const unsigned long long* hs, uint64_t rem, uint64_t& cum_out) {
    const int lane = threadIdx.x & 63;
    uint64_t h[4];
    uint64_t local = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        h[j] = hs[4 * lane + j];
        local += h[j];
    }
    uint64_t incl = local;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
    }
    uint64_t c = incl - local;
    int found = -1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (found < 0) {
            if (c + h[j] >= rem) found = 4 * lane + j;
            else c += h[j];
        }
    }
    const uint64_t bal = __ballot(found >= 0);
    if (bal == 0ull) return -1;
    const int src = __ffsll((long long)bal) - 1;
    cum_out = __shfl(c, src);
    return __shfl(found, src);
}

__global__ void k_trunc_keys(MatView X, const double* __restrict__ delta_dev, double delta_host, double scale,
                             TruncTemp t, int64_t cap, const int32_t* __restrict__ done) {
    if (done && *done) return;
    const double delta = (delta_dev ? *delta_dev : delta_host) * scale;
    const TruncQuanta q = trunc_quanta(delta);
    if (!q.any) return;
    int64_t nslot = *X.nslot;
    if (nslot > X.cap) nslot = X.cap;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslot; s += (int64_t)gridDim.x * blockDim.x) {
        const int r = X.brow[s];
        if (r < 0) continue;
        const int c = X.bcol[s];
        if (r > c) continue;
        const double w = (r == c) ? 1.0 : 2.0;
        const double v = w * X.sq[s];
        const double sc = v / q.Q;
        const uint64_t k = sc < (double)kKSat ? (uint64_t)ceil(sc) : kKSat;
        if (k < q.kt) {
            const uint64_t ukey = (uint64_t)r * (uint64_t)X.nb + (uint64_t)c;
            const unsigned long long pos = atomicAdd((unsigned long long*)t.ncand, 1ull);
            if ((int64_t)pos < cap) {
                t.key[pos] = (k << 22) | ukey;
                t.k[pos] = k;
            }
        }
    }
}

__global__ __launch_bounds__(1024) void k_trunc_select(const double* __restrict__ delta_dev, double delta_host,
                                                      double scale, TruncTemp t, int64_t cap, int32_t* __restrict__ ovf,
                                                      const int32_t* __restrict__ done) {
    __shared__ unsigned long long hs[256];
    __shared__ uint64_t s_prefix, s_rem, s_thr;
    __shared__ int s_fin;
    if (done && *done) return;
    const double delta = (delta_dev ? *delta_dev : delta_host) * scale;
    const TruncQuanta q = trunc_quanta(delta);
    int64_t n = *t.ncand;
    if (threadIdx.x == 0) {
        if (n > cap) atomicOr(ovf, kOvfCand);
        s_prefix = 0;
        s_rem = q.kt;
        s_thr = 0;
        s_fin = q.any ? 0 : 1;  // nothing removable
    }
    if (n > cap) n = cap;
    __syncthreads();
    for (int d = 0; d < 8; ++d) {
        if (s_fin) break;
        const int shift = 56 - 8 * d;
        const uint64_t mask_hi = d == 0 ? 0ull : ~((1ull << (shift + 8)) - 1ull);
        for (int b = threadIdx.x; b < 256; b += blockDim.x) hs[b] = 0ull;
        __syncthreads();
        const uint64_t pre = s_prefix;
        for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
            const uint64_t key = t.key[c];
            if ((key & mask_hi) == (pre & mask_hi))
                atomicAdd(&hs[(key >> shift) & 255u], (unsigned long long)t.k[c]);
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            uint64_t cum = 0;
            const int found = radix_bucket(hs, s_rem, cum);
            if (threadIdx.x == 0 && found < 0) {
                // every remaining unit in this range fits: remove the whole range
                s_thr = d == 0 ? ~0ull : ((pre | ((1ull << (shift + 8)) - 1ull)) + 1ull);
                s_fin = 1;
            } else if (threadIdx.x == 0) {
                s_prefix = pre | ((uint64_t)found << shift);
                s_rem = s_rem - cum;
                if (d == 7) {
                    s_thr = s_prefix;  // key of the first unit that does not fit
                    s_fin = 1;
                }
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *t.thr = q.any ? s_thr : 0ull;
}

__global__ void k_trunc_mark(MatView X, TruncTemp t, int64_t cap, int64_t* __restrict__ stats,
                             const int32_t* __restrict__ done) {
    if (done && *done) return;
    int64_t n = *t.ncand;
    if (n > cap) n = cap;
    const uint64_t thr = *t.thr;
    const int nb = X.nb;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = t.key[c];
        if (key >= thr) continue;
        const uint64_t ukey = key & ((1ull << 22) - 1ull);
        const int r = (int)(ukey / (uint64_t)nb), cc = (int)(ukey % (uint64_t)nb);
        const int s1 = X.map[(size_t)r * nb + cc];
        const int s2 = X.map[(size_t)cc * nb + r];
        if (s1 >= 0) X.brow[s1] = -1;
        if (s2 >= 0) X.brow[s2] = -1;
        const int nrem = (s1 >= 0 ? 1 : 0) + (s2 >= 0 && s2 != s1 ? 1 : 0);
        X.map[(size_t)r * nb + cc] = -1;
        X.map[(size_t)cc * nb + r] = -1;
        if (stats) {
            atomicAdd((unsigned long long*)&stats[0], 1ull);
            atomicAdd((unsigned long long*)&stats[1], (unsigned long long)t.k[c]);
            atomicAdd((unsigned long long*)&stats[2], (unsigned long long)nrem);
        }
    }
}

__global__ void k_trunc_reset(TruncTemp t, int64_t* stats, const int32_t* __restrict__ done) {
    if (done && *done) return;
    if (threadIdx.x == 0) {
        *t.ncand = 0;
        *t.thr = 0;
        if (stats) { stats[0] = 0; stats[1] = 0; stats[2] = 0; }
    }
}

// Small iterates (at most kTruncSmallCap slots): k_trunc_reset, k_trunc_keys,
// k_trunc_select and k_trunc_mark in one workgroup with the candidate keys in
// LDS (a candidate's k is its key >> 22).  Same quanta, keys and radix
// select, so the removed set and the statistics are the same.
__global__ __launch_bounds__(1024) void k_trunc_small(MatView X, const double* __restrict__ delta_dev,
                                                     double delta_host, double scale, int64_t* __restrict__ stats,
                                                     const int32_t* __restrict__ done) {
    __shared__ uint64_t s_key[kTruncSmallCap];
    __shared__ unsigned long long hs[256];
    __shared__ unsigned long long s_st[3];
    __shared__ uint64_t s_prefix, s_rem, s_thr;
    __shared__ int s_fin, s_n;
    if (done && *done) return;
    const int tid = threadIdx.x;
    const double delta = (delta_dev ? *delta_dev : delta_host) * scale;
    const TruncQuanta q = trunc_quanta(delta);
    if (tid == 0) {
        s_n = 0;
        s_st[0] = s_st[1] = s_st[2] = 0ull;
        s_prefix = 0;
        s_rem = q.kt;
        s_thr = 0;
        s_fin = q.any ? 0 : 1;
    }
    __syncthreads();
    int64_t nslot = *X.nslot;
    if (nslot > X.cap) nslot = X.cap;
    if (q.any) {
        for (int64_t s = tid; s < nslot; s += blockDim.x) {
            const int r = X.brow[s];
            if (r < 0) continue;
            const int c = X.bcol[s];
            if (r > c) continue;
            const double w = (r == c) ? 1.0 : 2.0;
            const double v = w * X.sq[s];
            const double sc = v / q.Q;
            const uint64_t k = sc < (double)kKSat ? (uint64_t)ceil(sc) : kKSat;
            if (k < q.kt) s_key[atomicAdd(&s_n, 1)] = (k << 22) | ((uint64_t)r * (uint64_t)X.nb + (uint64_t)c);
        }
    }
    __syncthreads();
    const int n = s_n;
    for (int d = 0; d < 8; ++d) {
        if (s_fin) break;
        const int shift = 56 - 8 * d;
        const uint64_t mask_hi = d == 0 ? 0ull : ~((1ull << (shift + 8)) - 1ull);
        for (int b = tid; b < 256; b += blockDim.x) hs[b] = 0ull;
        __syncthreads();
        const uint64_t pre = s_prefix;
        for (int c = tid; c < n; c += blockDim.x) {
            const uint64_t key = s_key[c];
            if ((key & mask_hi) == (pre & mask_hi)) atomicAdd(&hs[(key >> shift) & 255u], key >> 22);
        }
        __syncthreads();
        if (tid < 64) {
            uint64_t cum = 0;
            const int found = radix_bucket(hs, s_rem, cum);
            if (tid == 0 && found < 0) {
                s_thr = d == 0 ? ~0ull : ((pre | ((1ull << (shift + 8)) - 1ull)) + 1ull);
                s_fin = 1;
            } else if (threadIdx.x == 0) {
                s_prefix = pre | ((uint64_t)found << shift);
                s_rem = s_rem - cum;
                if (d == 7) {
                    s_thr = s_prefix;
                    s_fin = 1;
                }
            }
        }
        __syncthreads();
    }
    const uint64_t thr = q.any ? s_thr : 0ull;
    const int nb = X.nb;
    for (int c = tid; c < n; c += blockDim.x) {
        const uint64_t key = s_key[c];
        if (key >= thr) continue;
        const uint64_t ukey = key & ((1ull << 22) - 1ull);
        const int r = (int)(ukey / (uint64_t)nb), cc = (int)(ukey % (uint64_t)nb);
        const int s1 = X.map[(size_t)r * nb + cc];
        const int s2 = X.map[(size_t)cc * nb + r];
        if (s1 >= 0) X.brow[s1] = -1;
        if (s2 >= 0) X.brow[s2] = -1;
        const int nrem = (s1 >= 0 ? 1 : 0) + (s2 >= 0 && s2 != s1 ? 1 : 0);
        X.map[(size_t)r * nb + cc] = -1;
        X.map[(size_t)cc * nb + r] = -1;
        if (stats) {
            atomicAdd(&s_st[0], 1ull);
            atomicAdd(&s_st[1], (unsigned long long)(key >> 22));
            atomicAdd(&s_st[2], (unsigned long long)nrem);
        }
    }
    __syncthreads();
    if (stats && tid == 0) {
        stats[0] = (int64_t)s_st[0];
        stats[1] = (int64_t)s_st[1];
        stats[2] = (int64_t)s_st[2];
    }
}

// Scratch of the allocation-free truncation (spamm_truncate_noalloc): the
// candidate keys of up to kTruncNoallocMaxCap slots, then the removal
// statistics and the overflow word.  One copy per GPU, held until the process
// ends; every call on a GPU reuses it (the kernels clear what must start at
// zero), so calls that overlap on one GPU race.
constexpr int64_t kTruncNoallocMaxCap = (int64_t)1 << 20;
constexpr size_t kTruncNoallocStatsOff = ((size_t)kTruncNoallocMaxCap * 16 + 64 + 255) & ~(size_t)255;
constexpr size_t kTruncNoallocBytes = kTruncNoallocStatsOff + 256;
static __device__ __align__(256) char scratch[kTruncNoallocBytes];

int64_t trunc_noalloc_max_cap() { return kTruncNoallocMaxCap; }

// Device address of `scratch` on the current device, looked up once per
// device with that device current (the host-side name is not a device address).
hipError_t trunc_noalloc_scratch(TruncNoallocScratch* out) {
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static void* ptr[kMaxDev] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        ptr[dev] = p;
    }
    char* base = (char*)ptr[dev];
    out->temp = base;
    out->stats = (int64_t*)(base + kTruncNoallocStatsOff);
    out->ovf = (int32_t*)(base + kTruncNoallocStatsOff + 64);
    return hipSuccess;
}

void launch_truncate(const MatView& X, const double* delta_dev, double delta_host, double delta_scale, void* temp,
                     int64_t cap, int64_t* stats, int32_t* ovf, const int32_t* done, hipStream_t s) {
    if (X.cap <= kTruncSmallCap && small_path_enabled()) {
        hipLaunchKernelGGL(k_trunc_small, dim3(1), dim3(1024), 0, s, X, delta_dev, delta_host, delta_scale, stats,
                           done);
        return;
    }
    TruncTemp t = carve_trunc(temp, cap);
    hipLaunchKernelGGL(k_trunc_reset, dim3(1), dim3(64), 0, s, t, stats, done);
    hipLaunchKernelGGL(k_trunc_keys, dim3(grid_for(X.cap, 256, 4096)), dim3(256), 0, s, X, delta_dev, delta_host,
                       delta_scale, t, cap, done);
    hipLaunchKernelGGL(k_trunc_select, dim3(1), dim3(1024), 0, s, delta_dev, delta_host, delta_scale, t, cap, ovf,
                       done);
    hipLaunchKernelGGL(k_trunc_mark, dim3(grid_for(cap, 256, 4096)), dim3(256), 0, s, X, t, cap, stats, done);
}

}  // namespace spamm
