// Shared device helpers and launcher declarations of the gfx950 SpAMM
// library.  Everything in here is internal; the C ABI lives in api.hip and
// include/spamm.h.
#pragma once
#include <hip/hip_runtime.h>
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
};

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
