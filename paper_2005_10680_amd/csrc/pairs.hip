// Kept-pair enumeration for Algorithm 2 at the leaf level and the output
// pattern of the combined product.
//
// Row bitmaps of A (bit k of row i when A_ik is present) and column bitmaps
// of B (bit k of column j when B_kj is present) turn the candidate inner
// indices of output (i, j) into a word-wise AND.  Outputs are visited in
// 2D Morton order, so after the scans the output list, the kept-pair list
// and the slots of the result are all laid out along the linearised
// quadtree.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

__global__ void k_occupancy(MatView M, int mode, uint32_t* __restrict__ bits, int nw, uint8_t* __restrict__ tiles,
                            int T, int l0, const int32_t* __restrict__ done) {
    if (done && *done) return;
    int64_t nslot = *M.nslot;
    if (nslot > M.cap) nslot = M.cap;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslot; s += (int64_t)gridDim.x * blockDim.x) {
        int r = M.brow[s];
        if (r < 0) continue;
        int c = M.bcol[s];
        if (r >= M.nb || c < 0 || c >= M.nb) continue;
        int br, bit, tr, tc;
        if (mode == kOccA) { br = r; bit = c; tr = r; tc = c; }
        else if (mode == kOccB) { br = c; bit = r; tr = r; tc = c; }
        else { br = r; bit = c; tr = c; tc = r; }
        if (bits) atomicOr(&bits[(size_t)br * nw + (bit >> 5)], 1u << (bit & 31));
        if (tiles) tiles[(size_t)(tr >> l0) * T + (tc >> l0)] = 1;
    }
}

void launch_occupancy(const MatView& M, int mode, uint32_t* bits, int nw, uint8_t* tiles, int T, int l0,
                      const int32_t* done, hipStream_t s) {
    hipLaunchKernelGGL(k_occupancy, dim3(grid_for(M.cap, 256, 2048)), dim3(256), 0, s, M, mode, bits, nw, tiles, T,
                       l0, done);
}


// Eight lanes per output (i, j): lane g of the group walks the contiguous
// bitmap words [g nw / 8, (g + 1) nw / 8) of the candidate inner indices, so
// an output's map and norm loads run on eight lanes at once rather than one
// after another; the lanes hold ascending k ranges in lane order.
constexpr int kKeptG = 8;

// kept pairs (and low-tier pairs) of output (i, j) in this lane's words
SPAMM_DEV void kept_lane_count(int i, int j, int w0, int w1, int nb, int nw, const uint32_t* __restrict__ bitsA,
                               const uint32_t* __restrict__ bitsB, const int32_t* __restrict__ mapA,
                               const double* __restrict__ normA, const int32_t* __restrict__ mapB,
                               const double* __restrict__ normB, int btrans, double tau, double sigma,
                               double norm_min, int& c, int& cl) {
    c = 0;
    cl = 0;
    for (int w = w0; w < w1; ++w) {
        uint32_t m = bitsA[(size_t)i * nw + w] & bitsB[(size_t)j * nw + w];
        while (m) {
            const int k = w * 32 + __ffs(m) - 1;
            m &= m - 1;
            const int sa = mapA[(size_t)i * nb + k];
            const int sb = btrans ? mapB[(size_t)j * nb + k] : mapB[(size_t)k * nb + j];
            if (sa < 0 || sb < 0) continue;
            const double p = normA[sa] * normB[sb];
            if (!(p >= tau)) continue;
            ++c;
            if (p < sigma && normA[sa] >= norm_min && normB[sb] >= norm_min) ++cl;
        }
    }
}

__global__ void k_kept_count(int nb, int P, int nw, const uint32_t* __restrict__ bitsA,
                             const uint32_t* __restrict__ bitsB, const int32_t* __restrict__ mapA,
                             const double* __restrict__ normA, const int32_t* __restrict__ mapB,
                             const double* __restrict__ normB, int btrans, int sym, const double* __restrict__ tau_p,
                             const double* __restrict__ sigma_p, double norm_min, int32_t* __restrict__ cnt,
                             int32_t* __restrict__ cnt_flag, int32_t* __restrict__ cnt_low,
                             const int32_t* __restrict__ done) {
    if (done && *done) return;
    const double tau = *tau_p;
    const double sigma = sigma_p ? *sigma_p : 0.0;
    const int64_t PP = (int64_t)P * P;
    const int g = threadIdx.x % kKeptG;
    const int w0 = g * nw / kKeptG, w1 = (g + 1) * nw / kKeptG;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kKeptG);
    // z is uniform over the eight lanes of a group (blockDim.x is a multiple of 8)
    for (int64_t z = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kKeptG; z < PP; z += groups) {
        uint32_t i, j;
        demorton2((uint32_t)z, i, j);
        int c = 0, cl = 0;
        if ((int)i < nb && (int)j < nb && !(sym && i > j))
            kept_lane_count((int)i, (int)j, w0, w1, nb, nw, bitsA, bitsB, mapA, normA, mapB, normB, btrans, tau,
                            sigma, norm_min, c, cl);
#pragma unroll
        for (int d = 1; d < kKeptG; d <<= 1) {
            c += __shfl_xor(c, d, kKeptG);
            cl += __shfl_xor(cl, d, kKeptG);
        }
        if (g == 0) {
            cnt[z] = c;
            cnt_flag[z] = c > 0 ? 1 : 0;
            if (cnt_low) cnt_low[z] = cl;
        }
    }
}

void launch_kept_count(int nb, int P, int nw, const uint32_t* bitsA, const uint32_t* bitsB, const int32_t* mapA,
                       const double* normA, const int32_t* mapB, const double* normB, int btrans, int sym,
                       const double* tau, const double* sigma, double norm_min, int32_t* cnt, int32_t* cnt_flag,
                       int32_t* cnt_low, const int32_t* done, hipStream_t s) {
    int64_t PP = (int64_t)P * P;
    hipLaunchKernelGGL(k_kept_count, dim3(grid_for(PP * kKeptG, 256, 8192)), dim3(256), 0, s, nb, P, nw, bitsA, bitsB,
                       mapA, normA, mapB, normB, btrans, sym, tau, sigma, norm_min, cnt, cnt_flag, cnt_low, done);
}

// Pairs of one output: low-precision pairs (tau <= p < sigma, both block
// norms >= norm_min) first, then the FP64 ones, each group in ascending k.
// Without tiers (sigma null) every pair is FP64.  Each lane of the output's
// group counts its words' pairs of both kinds, the group's exclusive scans
// (in lane order, i.e. ascending k) give the lane's first position in each
// part, and a second walk writes them.
__global__ void k_kept_fill(int nb, int P, int nw, const uint32_t* __restrict__ bitsA,
                            const uint32_t* __restrict__ bitsB, const int32_t* __restrict__ mapA,
                            const double* __restrict__ normA, const int32_t* __restrict__ mapB,
                            const double* __restrict__ normB, int btrans, const double* __restrict__ tau_p,
                            const double* __restrict__ sigma_p, double norm_min, const int32_t* __restrict__ cnt,
                            const int32_t* __restrict__ off, const int32_t* __restrict__ oidx,
                            const int64_t* __restrict__ npairs_p, const int64_t* __restrict__ nout_p, int64_t cap_pairs,
                            int64_t cap_out, int32_t* __restrict__ oi, int32_t* __restrict__ oj,
                            int32_t* __restrict__ optr, int2* __restrict__ pairs, int32_t* __restrict__ olow,
                            int32_t* __restrict__ ovf, const int32_t* __restrict__ done) {
    if (done && *done) return;
    const double tau = *tau_p;
    // without tiers no pair is low (sigma 0: p < 0 never holds for a kept p >= tau >= 0)
    const double sigma = sigma_p ? *sigma_p : 0.0;
    const int64_t PP = (int64_t)P * P;
    const int64_t npairs = *npairs_p, nout = *nout_p;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (nout <= cap_out) optr[nout] = (int32_t)(npairs <= cap_pairs ? npairs : cap_pairs);
        if (npairs > cap_pairs) atomicOr(ovf, kOvfPairs);
        if (nout > cap_out) atomicOr(ovf, kOvfOut);
    }
    // an overflowing list is reported, not filled (its 32-bit offsets may have wrapped)
    if (npairs > cap_pairs) return;
    const int g = threadIdx.x % kKeptG;
    const int w0 = g * nw / kKeptG, w1 = (g + 1) * nw / kKeptG;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kKeptG);
    for (int64_t z = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kKeptG; z < PP; z += groups) {
        if (cnt[z] == 0) continue;  // group-uniform
        uint32_t i, j;
        demorton2((uint32_t)z, i, j);
        const int64_t o = oidx[z];
        if (o >= cap_out) continue;
        int c = 0, cl = 0;
        kept_lane_count((int)i, (int)j, w0, w1, nb, nw, bitsA, bitsB, mapA, normA, mapB, normB, btrans, tau, sigma,
                        norm_min, c, cl);
        const int ch = c - cl;
        // inclusive scans over the group's lanes, then exclusive
        int sl = cl, sh = ch;
#pragma unroll
        for (int d = 1; d < kKeptG; d <<= 1) {
            const int ul = __shfl_up(sl, d, kKeptG), uh = __shfl_up(sh, d, kKeptG);
            if (g >= d) {
                sl += ul;
                sh += uh;
            }
        }
        const int low_tot = __shfl(sl, kKeptG - 1, kKeptG);
        const int64_t base = off[z];
        int64_t wl = base + (sl - cl);             // this lane's first low-tier pair
        int64_t wh = base + low_tot + (sh - ch);   // this lane's first FP64 pair
        if (g == 0) {
            oi[o] = (int32_t)i;
            oj[o] = (int32_t)j;
            optr[o] = (int32_t)base;
            if (sigma_p && olow) olow[o] = low_tot;
        }
        if (c == 0) continue;
        for (int w = w0; w < w1; ++w) {
            uint32_t m = bitsA[(size_t)i * nw + w] & bitsB[(size_t)j * nw + w];
            while (m) {
                const int k = w * 32 + __ffs(m) - 1;
                m &= m - 1;
                const int sa = mapA[(size_t)i * nb + k];
                const int sb = btrans ? mapB[(size_t)j * nb + k] : mapB[(size_t)k * nb + j];
                if (sa < 0 || sb < 0) continue;
                const double p = normA[sa] * normB[sb];
                if (!(p >= tau)) continue;
                const bool low = p < sigma && normA[sa] >= norm_min && normB[sb] >= norm_min;
                const int64_t wp = low ? wl : wh;
                if (wp < cap_pairs) pairs[wp] = make_int2(sa, sb);
                if (low) ++wl;
                else ++wh;
            }
        }
    }
}

void launch_kept_fill(int nb, int P, int nw, const uint32_t* bitsA, const uint32_t* bitsB, const int32_t* mapA,
                      const double* normA, const int32_t* mapB, const double* normB, int btrans, const double* tau,
                      const double* sigma, double norm_min, const int32_t* cnt, const int32_t* off,
                      const int32_t* oidx, const int64_t* npairs, const int64_t* nout, int64_t cap_pairs,
                      int64_t cap_out, int32_t* oi, int32_t* oj, int32_t* optr, int2* pairs, int32_t* olow,
                      int32_t* ovf, const int32_t* done, hipStream_t s) {
    int64_t PP = (int64_t)P * P;
    hipLaunchKernelGGL(k_kept_fill, dim3(grid_for(PP * kKeptG, 256, 8192)), dim3(256), 0, s, nb, P, nw, bitsA, bitsB,
                       mapA, normA, mapB, normB, btrans, tau, sigma, norm_min, cnt, off, oidx, npairs, nout, cap_pairs,
                       cap_out, oi, oj, optr, pairs, olow, ovf, done);
}

// Output pattern: block (r, c) of the result exists when the product has a
// kept pair there (its upper-triangle mirror in symmetric mode) or, in the
// 2X - X^2 branch, when X has the block.
__global__ void k_hat_flags(int nb, int P, const int32_t* __restrict__ cnt, int sym, const int32_t* __restrict__ mapX,
                            const int32_t* __restrict__ branch, int32_t* __restrict__ flag,
                            const int32_t* __restrict__ done) {
    if (done && *done) return;
    const int br = branch ? *branch : 0;
    const int64_t PP = (int64_t)P * P;
    for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < PP; z += (int64_t)gridDim.x * blockDim.x) {
        uint32_t r, c;
        demorton2((uint32_t)z, r, c);
        int f = 0;
        if ((int)r < nb && (int)c < nb) {
            uint32_t cz = sym ? morton2(min(r, c), max(r, c)) : (uint32_t)z;
            f = cnt[cz] > 0;
            if (!f && mapX && br == 1) f = mapX[(size_t)r * nb + c] >= 0;
        }
        flag[z] = f;
    }
}

void launch_hat_flags(int nb, int P, const int32_t* cnt, int sym, const int32_t* mapX, const int32_t* branch,
                      int32_t* flag, const int32_t* done, hipStream_t s) {
    int64_t PP = (int64_t)P * P;
    hipLaunchKernelGGL(k_hat_flags, dim3(grid_for(PP, 256, 8192)), dim3(256), 0, s, nb, P, cnt, sym, mapX, branch,
                       flag, done);
}

__global__ void k_hat_assign(int nb, int P, const int32_t* __restrict__ cnt, int sym, const int32_t* __restrict__ flag,
                             const int32_t* __restrict__ slot, const int64_t* __restrict__ total, int64_t cap,
                             int32_t* __restrict__ map, int32_t* __restrict__ brow, int32_t* __restrict__ bcol,
                             int32_t* __restrict__ nslot, uint8_t* __restrict__ fromc, int32_t* __restrict__ ovf,
                             const int32_t* __restrict__ done) {
    if (done && *done) return;
    const int64_t PP = (int64_t)P * P;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t t = *total;
        *nslot = (int32_t)(t <= cap ? t : cap);
        if (t > cap) atomicOr(ovf, kOvfSlots);
    }
    for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < PP; z += (int64_t)gridDim.x * blockDim.x) {
        uint32_t r, c;
        demorton2((uint32_t)z, r, c);
        if ((int)r >= nb || (int)c >= nb) continue;
        int32_t m = -1;
        if (flag[z]) {
            int64_t sl = slot[z];
            if (sl < cap) {
                m = (int32_t)sl;
                brow[sl] = (int32_t)r;
                bcol[sl] = (int32_t)c;
                uint32_t cz = sym ? morton2(min(r, c), max(r, c)) : (uint32_t)z;
                if (fromc) fromc[sl] = cnt[cz] > 0 ? 1 : 0;
            }
        }
        map[(size_t)r * nb + c] = m;
    }
}

void launch_hat_assign(int nb, int P, const int32_t* cnt, int sym, const int32_t* flag, const int32_t* slot,
                       const int64_t* nslot_total, int64_t cap, int32_t* map, int32_t* brow, int32_t* bcol,
                       int32_t* nslot, uint8_t* fromc, int32_t* ovf, const int32_t* done, hipStream_t s) {
    int64_t PP = (int64_t)P * P;
    hipLaunchKernelGGL(k_hat_assign, dim3(grid_for(PP, 256, 8192)), dim3(256), 0, s, nb, P, cnt, sym, flag, slot,
                       nslot_total, cap, map, brow, bcol, nslot, fromc, ovf, done);
}

// Blocks of 2X - X^2 that no kept pair touches: X^ = 2 X (with their norms
// when no.sq is set, and their FP32 copies in the ring kernel's layout when
// out32 is).
template <int B>
__global__ __launch_bounds__(256) void k_rest(const int32_t* __restrict__ nslot_p, int64_t cap,
                                             const int32_t* __restrict__ brow, const int32_t* __restrict__ bcol,
                                             const uint8_t* __restrict__ fromc, int nb, const int32_t* __restrict__ mapX,
                                             const double* __restrict__ valX, double* __restrict__ valH,
                                             const int32_t* __restrict__ branch, const int32_t* __restrict__ done,
                                             NormOut no, float* __restrict__ out32) {
    if (done && *done) return;
    if (*branch != 1) return;
    int64_t nslot = *nslot_p;
    if (nslot > cap) nslot = cap;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t s = (int64_t)blockIdx.x * 4 + wv; s < nslot; s += (int64_t)gridDim.x * 4) {
        int r = brow[s];
        if (r < 0 || fromc[s]) continue;
        int sx = mapX[(size_t)r * nb + bcol[s]];
        if (sx < 0) continue;
        const double2* src = reinterpret_cast<const double2*>(valX + (size_t)sx * B * B);
        double2* dst = reinterpret_cast<double2*>(valH + (size_t)s * B * B);
        float2* d32 = out32 ? reinterpret_cast<float2*>(out32 + (size_t)s * B * B) : nullptr;
        SqAcc a;
        for (int t = lane; t < B * B / 2; t += 64) {
            double2 v = src[t];
            v.x = 2.0 * v.x;
            v.y = 2.0 * v.y;
            dst[t] = v;
            if (no.sq) {
                sq_add(a, v.x);
                sq_add(a, v.y);
            }
            if (d32) {
                // element pair (m, m + 1) of row k, m even: stays a pair after the rotation
                const int k = (2 * t) / B, m = (2 * t) % B;
                d32[(k * B + ((m + f32_rot<B>(k)) & (B - 1))) / 2] = float2{(float)v.x, (float)v.y};
            }
        }
        if (no.sq) {
            const dd acc = dd_wave_sum(a.acc);
            const bool ok = sq_certified(acc, __any(a.special), __any(a.tiny));
            if (lane == 0) {
                if (ok) {
                    no.sq[s] = acc.hi;
                    no.sqlo[s] = acc.lo;
                    no.nrm[s] = sqrt(acc.hi);
                } else {
                    no.recheck[atomicAdd(no.nrecheck, 1)] = (int32_t)s;
                }
            }
        }
    }
}

void launch_rest(int b, const int32_t* nslot_hat, int64_t cap_hat, const int32_t* brow, const int32_t* bcol,
                 const uint8_t* fromc, int nb, const int32_t* mapX, const double* valX, double* valH,
                 const int32_t* branch, const int32_t* done, hipStream_t s, NormOut no, float* out32) {
    int grid = grid_for(cap_hat, 4, 4096);
    switch (b) {
        case 32: hipLaunchKernelGGL(k_rest<32>, dim3(grid), dim3(256), 0, s, nslot_hat, cap_hat, brow, bcol, fromc, nb, mapX, valX, valH, branch, done, no, out32); break;
        case 64: hipLaunchKernelGGL(k_rest<64>, dim3(grid), dim3(256), 0, s, nslot_hat, cap_hat, brow, bcol, fromc, nb, mapX, valX, valH, branch, done, no, out32); break;
        case 128: hipLaunchKernelGGL(k_rest<128>, dim3(grid), dim3(256), 0, s, nslot_hat, cap_hat, brow, bcol, fromc, nb, mapX, valX, valH, branch, done, no, nullptr); break;
    }
}

// ---------------------------------------------------------------------------
// Small systems (nb <= kSmallNb): the passes above, each chain of launches
// in one workgroup.  Same lists in the same order (exclusive scans in 2D
// Morton order of the outputs, ascending k inside an output), so the
// products, their norms and every later decision are bit-identical to the
// device-wide passes; only the number of dependent launches per step
// changes.
// ---------------------------------------------------------------------------
constexpr int kSmallThreads = 1024;
constexpr int kSmallPer = kSmallPP / kSmallThreads;
static_assert(kSmallPP % kSmallThreads == 0, "whole items per thread");

// Occupancy of a symmetric-pattern X (row bitmaps and level-l0 tiles, as
// k_occupancy with kOccA) built in LDS; then, with cube_keys given, the
// non-empty cubes of the sweep of X X^T (k_cube_flags, the scan and
// k_cube_list with A = B = X) in ascending 3D Morton order.
__global__ __launch_bounds__(kSmallThreads) void k_occ_small(MatView X, uint32_t* __restrict__ bits, int nw,
                                                             uint8_t* __restrict__ tiles, int T, int l0,
                                                             uint32_t* __restrict__ cube_keys,
                                                             int64_t* __restrict__ ncubes,
                                                             const int32_t* __restrict__ done) {
    __shared__ uint32_t s_bits[kSmallNb * ((kSmallNb + 31) / 32)];
    __shared__ uint8_t s_tiles[kSmallTiles * kSmallTiles];
    __shared__ int64_t s_wave[kSmallThreads / 64];
    if (done && *done) return;
    const int tid = threadIdx.x;
    const int nwords = X.nb * nw;
    for (int t = tid; t < nwords; t += kSmallThreads) s_bits[t] = 0u;
    for (int t = tid; t < T * T; t += kSmallThreads) s_tiles[t] = 0;
    __syncthreads();
    int64_t nslot = *X.nslot;
    if (nslot > X.cap) nslot = X.cap;
    for (int64_t s = tid; s < nslot; s += kSmallThreads) {
        const int r = X.brow[s];
        if (r < 0) continue;
        const int c = X.bcol[s];
        if (r >= X.nb || c < 0 || c >= X.nb) continue;
        atomicOr(&s_bits[r * nw + (c >> 5)], 1u << (c & 31));
        s_tiles[(r >> l0) * T + (c >> l0)] = 1;
    }
    __syncthreads();
    for (int t = tid; t < nwords; t += kSmallThreads) bits[t] = s_bits[t];
    for (int t = tid; t < T * T; t += kSmallThreads) tiles[t] = s_tiles[t];
    if (!cube_keys) return;
    // cubes: thread tid owns the kCubesPer consecutive Morton codes from tid * kCubesPer
    constexpr int kCubesPer = kSmallTiles * kSmallTiles * kSmallTiles / kSmallThreads;
    const int TTT = T * T * T;
    const int z0 = tid * kCubesPer;
    int f[kCubesPer];
    int nf = 0;
#pragma unroll
    for (int u = 0; u < kCubesPer; ++u) {
        f[u] = 0;
        if (z0 + u < TTT) {
            uint32_t I, K, J;
            demorton3((uint32_t)(z0 + u), I, K, J);
            f[u] = (s_tiles[I * T + K] && s_tiles[K * T + J]) ? 1 : 0;
        }
        nf += f[u];
    }
    int64_t tot = 0;
    int64_t pos = block_inclusive_scan<kSmallThreads>(nf, s_wave, tot) - nf;
#pragma unroll
    for (int u = 0; u < kCubesPer; ++u)
        if (f[u]) cube_keys[pos++] = (uint32_t)(z0 + u);
    if (tid == 0) *ncubes = tot;
}

void launch_occ_small(const MatView& X, uint32_t* bits, int nw, uint8_t* tiles, int T, int l0, uint32_t* cube_keys,
                      int64_t* ncubes, const int32_t* done, hipStream_t s) {
    hipLaunchKernelGGL(k_occ_small, dim3(1), dim3(kSmallThreads), 0, s, X, bits, nw, tiles, T, l0, cube_keys, ncubes,
                       done);
}

// k_kept_count, the scans of the counts, the output flags and the low-tier
// counts, k_kept_fill, k_hat_flags, the scan of the output pattern and
// k_hat_assign for P * P <= kSmallPP outputs; also clears the product's 16
// work counters (the product launch then skips its own reset).  Output z is
// taken by thread z mod kSmallThreads in round z / kSmallThreads, so small
// grids keep every thread busy; the three counts of an output travel packed
// in one 64-bit scan (21 bits each: at most 64 * 4096 pairs).
__global__ __launch_bounds__(kSmallThreads) void k_pairs_small(
    int nb, int P, int nw, const uint32_t* __restrict__ bitsA, const uint32_t* __restrict__ bitsB,
    const int32_t* __restrict__ mapA, const double* __restrict__ normA, const int32_t* __restrict__ mapB,
    const double* __restrict__ normB, int btrans, int sym, const double* __restrict__ tau_p,
    const double* __restrict__ sigma_p, double norm_min, int64_t cap_pairs, int64_t cap_out, int32_t* __restrict__ oi,
    int32_t* __restrict__ oj, int32_t* __restrict__ optr, int2* __restrict__ pairs, int32_t* __restrict__ olow,
    int64_t* __restrict__ sc, int64_t capC, int32_t* __restrict__ mapC, int32_t* __restrict__ browC,
    int32_t* __restrict__ bcolC, int32_t* __restrict__ nslotC, uint8_t* __restrict__ fromc,
    const int32_t* __restrict__ mapX, const int32_t* __restrict__ branch_p, int32_t* __restrict__ counters,
    int32_t* __restrict__ cuts, int32_t* __restrict__ ovf, const int32_t* __restrict__ done) {
    constexpr int kBits = 21;
    constexpr int64_t kMask = ((int64_t)1 << kBits) - 1;
    __shared__ int32_t s_cnt[kSmallPP];
    __shared__ int64_t s_wave[kSmallThreads / 64];
    __shared__ int32_t s_cut[8];
    if (done && *done) return;
    const int tid = threadIdx.x;
    if (tid < 16) counters[tid] = 0;
    if (tid < 8) s_cut[tid] = 0;
    const double tau = *tau_p;
    const double sigma = sigma_p ? *sigma_p : 0.0;
    const int PP = P * P;
    const int R = (PP + kSmallThreads - 1) / kSmallThreads;
    int64_t off[kSmallPer], oix[kSmallPer];
    int64_t base = 0;
#pragma unroll
    for (int u = 0; u < kSmallPer; ++u) {
        if (u >= R) break;
        const int z = u * kSmallThreads + tid;
        int c = 0, cl = 0;
        if (z < PP) {
            uint32_t i, j;
            demorton2((uint32_t)z, i, j);
            if ((int)i < nb && (int)j < nb && !(sym && i > j)) {
                for_each_kept((int)i, (int)j, nb, nw, bitsA, bitsB, mapA, normA, mapB, normB, btrans, tau,
                              [&](int, int sa, int sb, double p) {
                                  ++c;
                                  if (p < sigma && normA[sa] >= norm_min && normB[sb] >= norm_min) ++cl;
                              });
            }
            s_cnt[z] = c;
        }
        const int64_t v = (int64_t)c | ((int64_t)(c > 0 ? 1 : 0) << kBits) | ((int64_t)cl << (2 * kBits));
        int64_t tot = 0;
        const int64_t ex = base + block_inclusive_scan<kSmallThreads>(v, s_wave, tot) - v;
        off[u] = ex & kMask;
        oix[u] = (ex >> kBits) & kMask;
        base += tot;
    }
    const int64_t npairs = base & kMask, nout = (base >> kBits) & kMask, nlow = base >> (2 * kBits);
    if (tid == 0) {
        sc[0] = npairs;
        sc[1] = nout;
        sc[3] = sigma_p ? nlow : 0;
        if (nout <= cap_out) optr[nout] = (int32_t)(npairs <= cap_pairs ? npairs : cap_pairs);
        if (npairs > cap_pairs) atomicOr(ovf, kOvfPairs);
        if (nout > cap_out) atomicOr(ovf, kOvfOut);
    }
    // kept pairs of each output: low tier first, then FP64, ascending k in
    // each; and the product's per-XCD output ranges (k_gemm_ring's cut x:
    // the outputs whose first pair lies below npairs * x / 8)
    if (npairs <= cap_pairs) {
#pragma unroll
        for (int u = 0; u < kSmallPer; ++u) {
            if (u >= R) break;
            const int z = u * kSmallThreads + tid;
            if (z >= PP || s_cnt[z] == 0) continue;
            const int64_t o = oix[u];
            if (o >= cap_out) continue;
            uint32_t i, j;
            demorton2((uint32_t)z, i, j);
            oi[o] = (int32_t)i;
            oj[o] = (int32_t)j;
            optr[o] = (int32_t)off[u];
            for (int x = 1; x < 8; ++x)
                if (off[u] < npairs * x / 8) atomicAdd(&s_cut[x], 1);
            int64_t w = off[u];
            if (sigma_p) {
                for_each_kept((int)i, (int)j, nb, nw, bitsA, bitsB, mapA, normA, mapB, normB, btrans, tau,
                              [&](int, int sa, int sb, double p) {
                                  if (p < sigma && normA[sa] >= norm_min && normB[sb] >= norm_min) {
                                      if (w < cap_pairs) pairs[w] = make_int2(sa, sb);
                                      ++w;
                                  }
                              });
                if (olow) olow[o] = (int32_t)(w - off[u]);
                for_each_kept((int)i, (int)j, nb, nw, bitsA, bitsB, mapA, normA, mapB, normB, btrans, tau,
                              [&](int, int sa, int sb, double p) {
                                  if (!(p < sigma && normA[sa] >= norm_min && normB[sb] >= norm_min)) {
                                      if (w < cap_pairs) pairs[w] = make_int2(sa, sb);
                                      ++w;
                                  }
                              });
            } else {
                for_each_kept((int)i, (int)j, nb, nw, bitsA, bitsB, mapA, normA, mapB, normB, btrans, tau,
                              [&](int, int sa, int sb, double) {
                                  if (w < cap_pairs) pairs[w] = make_int2(sa, sb);
                                  ++w;
                              });
            }
        }
    }
    // output pattern (k_hat_flags) and its slots (k_hat_assign)
    const int br = branch_p ? *branch_p : 0;
    int64_t hbase = 0;
#pragma unroll
    for (int u = 0; u < kSmallPer; ++u) {
        if (u >= R) break;
        const int z = u * kSmallThreads + tid;
        uint32_t r = 0, c = 0;
        int hf = 0;
        bool in = false;
        if (z < PP) {
            demorton2((uint32_t)z, r, c);
            in = (int)r < nb && (int)c < nb;
            if (in) {
                const uint32_t cz = sym ? morton2(min(r, c), max(r, c)) : (uint32_t)z;
                hf = s_cnt[cz] > 0;
                if (!hf && mapX && br == 1) hf = mapX[(size_t)r * nb + c] >= 0;
            }
        }
        int64_t tot = 0;
        const int64_t sl = hbase + block_inclusive_scan<kSmallThreads>(hf, s_wave, tot) - hf;
        hbase += tot;
        if (in) {
            int32_t m = -1;
            if (hf && sl < capC) {
                m = (int32_t)sl;
                browC[sl] = (int32_t)r;
                bcolC[sl] = (int32_t)c;
                const uint32_t cz = sym ? morton2(min(r, c), max(r, c)) : (uint32_t)z;
                if (fromc) fromc[sl] = s_cnt[cz] > 0 ? 1 : 0;
            }
            mapC[(size_t)r * nb + c] = m;
        }
    }
    __syncthreads();
    if (tid == 0) {
        sc[2] = hbase;
        *nslotC = (int32_t)(hbase <= capC ? hbase : capC);
        if (hbase > capC) atomicOr(ovf, kOvfSlots);
    }
    if (cuts && tid < 9) cuts[tid] = tid == 8 ? (int32_t)nout : s_cut[tid];
}

void launch_pairs_small(int nb, int P, int nw, const uint32_t* bitsA, const uint32_t* bitsB, const int32_t* mapA,
                        const double* normA, const int32_t* mapB, const double* normB, int btrans, int sym,
                        const double* tau, const double* sigma, double norm_min, int64_t cap_pairs, int64_t cap_out,
                        int32_t* oi, int32_t* oj, int32_t* optr, int2* pairs, int32_t* olow, int64_t* sc,
                        int64_t capC, int32_t* mapC, int32_t* browC, int32_t* bcolC, int32_t* nslotC,
                        uint8_t* fromc, const int32_t* mapX, const int32_t* branch, int32_t* counters,
                        int32_t* cuts, int32_t* ovf, const int32_t* done, hipStream_t s) {
    hipLaunchKernelGGL(k_pairs_small, dim3(1), dim3(kSmallThreads), 0, s, nb, P, nw, bitsA, bitsB, mapA, normA, mapB,
                       normB, btrans, sym, tau, sigma, norm_min, cap_pairs, cap_out, oi, oj, optr, pairs, olow, sc,
                       capC, mapC, browC, bcolC, nslotC, fromc, mapX, branch, counters, cuts, ovf, done);
}

}  // namespace spamm
