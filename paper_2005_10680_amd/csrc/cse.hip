// K2: the error-bound sweep (Algorithm 3, CSE) for every candidate
// threshold at once, and the selection rule.
//
// The product recursion of Algorithm 3 is an octree over (i, k, j) block
// triples.  Nodes are identified by 3D Morton keys, whose low three bits are
// the octant (a, kappa, c) inside the parent.  The bottom l0 levels are
// evaluated per "cube" (2^l0 x 2^l0 x 2^l0 triples): the cube's A and B
// leaf norms are staged in LDS and each candidate's subtree is walked in the
// canonical order of Algorithm 3 (a = row half outer, c = column half inner,
// t = E1 + E2, acc += t^2, sqrt at the end) -- by one thread when there are
// few candidates (several cubes per workgroup), else by eight threads, one
// per child subtree, one of them then combining the eight in the same
// order.  The levels above run as segmented reductions over the
// sorted node lists, one launch per level.  All arithmetic is in the
// paper's order with one rounding per operation, so every candidate's bound
// is bit-identical to the recursive definition.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

static int ceil_log2(int x) {
    int L = 0;
    while ((1 << L) < x) ++L;
    return L;
}

int cse_level0(int nb) {
    int L = ceil_log2(nb);
    int l0 = L - 7;  // at most 128^3 cubes
    if (l0 < 3) l0 = 3;
    if (l0 > L) l0 = L;
    return l0;
}

size_t cse_cube_cap(int nb) {
    int L = ceil_log2(nb);
    int T = 1 << (L - cse_level0(nb));
    return (size_t)T * T * T;
}

__global__ void k_cube_flags(int T, const uint8_t* __restrict__ tA, const uint8_t* __restrict__ tB,
                             int32_t* __restrict__ flag, const int32_t* __restrict__ done) {
    if (done && *done) return;
    const int64_t TTT = (int64_t)T * T * T;
    for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < TTT; z += (int64_t)gridDim.x * blockDim.x) {
        uint32_t I, K, J;
        demorton3((uint32_t)z, I, K, J);
        flag[z] = (tA[(size_t)I * T + K] && tB[(size_t)K * T + J]) ? 1 : 0;
    }
}

void launch_cube_flags(int T, const uint8_t* tilesA, const uint8_t* tilesB, int32_t* flag, const int32_t* done,
                       hipStream_t s) {
    int64_t TTT = (int64_t)T * T * T;
    hipLaunchKernelGGL(k_cube_flags, dim3(grid_for(TTT, 256, 8192)), dim3(256), 0, s, T, tilesA, tilesB, flag, done);
}

__global__ void k_cube_list(int T, const int32_t* __restrict__ flag, const int32_t* __restrict__ idx,
                            uint32_t* __restrict__ keys, const int64_t* __restrict__ ncubes, int64_t cap,
                            int32_t* __restrict__ ovf, const int32_t* __restrict__ done) {
    if (done && *done) return;
    const int64_t TTT = (int64_t)T * T * T;
    if (blockIdx.x == 0 && threadIdx.x == 0 && *ncubes > cap) atomicOr(ovf, kOvfCubes);
    for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < TTT; z += (int64_t)gridDim.x * blockDim.x) {
        if (flag[z] && idx[z] < cap) keys[idx[z]] = (uint32_t)z;
    }
}

void launch_cube_list(int T, const int32_t* flag, const int32_t* idx, uint32_t* keys, const int64_t* ncubes,
                      int64_t cap, int32_t* ovf, const int32_t* done, hipStream_t s) {
    int64_t TTT = (int64_t)T * T * T;
    hipLaunchKernelGGL(k_cube_list, dim3(grid_for(TTT, 256, 8192)), dim3(256), 0, s, T, flag, idx, keys, ncubes, cap,
                       ovf, done);
}

// Error of the subtree rooted at level LEV, node (i0, k0, j0) inside the
// cube; P holds the cube's leaf products p = RN(nu(A_ik) nu(B_kj)) at
// (i * S + k) * S + j.
template <int LEV, int S, int MODE>
SPAMM_DEV double cube_node(int i0, int k0, int j0, double tm, double t0, double cl, const double* P) {
    if constexpr (LEV == 0) {
        const double p = P[(i0 * S + k0) * S + j0];
        if constexpr (MODE == 0) {
            return p < tm ? p : 0.0;
        } else {
            return p < t0 ? p : (p < tm ? cl * p : 0.0);
        }
    } else {
        // canonical order: a (row half) outer, c (column half) inner; only the
        // two children of the current (a, c) are live, so the levels above the
        // first are left rolled to keep the recursion in registers
        double acc = 0.0;
#pragma unroll(LEV == 1 ? 2 : 1)
        for (int a = 0; a < 2; ++a)
#pragma unroll(LEV == 1 ? 2 : 1)
            for (int c = 0; c < 2; ++c) {
                double e1 = cube_node<LEV - 1, S, MODE>(2 * i0 + a, 2 * k0, 2 * j0 + c, tm, t0, cl, P);
                double e2 = cube_node<LEV - 1, S, MODE>(2 * i0 + a, 2 * k0 + 1, 2 * j0 + c, tm, t0, cl, P);
                double t = e1 + e2;
                double t2 = t * t;
                acc = acc + t2;
            }
        return sqrt(acc);
    }
}

// LDS for the leaf products of the cubes of one workgroup (doubles)
constexpr int kCubeLds = 4096;

// Few candidates (N <= 64): workgroups of 256 threads take `cpw` cubes at a
// time, `lpc` threads per cube (candidates m = lane, lane + lpc, ...): the
// leaf norms of the cubes go to LDS, then their S^3 leaf products (computed
// once, shared by every candidate), then each thread evaluates Algorithm 3
// over its cube for its candidates.
template <int L0, int MODE>
__global__ __launch_bounds__(256) void k_cube_eval_whole(int nb, const uint32_t* __restrict__ keys,
                                                  const int64_t* __restrict__ ncubes_p, int64_t cap,
                                                  const int32_t* __restrict__ mapA, const double* __restrict__ normA,
                                                  const int32_t* __restrict__ mapB, const double* __restrict__ normB,
                                                  int btrans, const double* __restrict__ tau, int N,
                                                  const double* __restrict__ tau0_p, double c_low, int cpw, int lpc,
                                                  double* __restrict__ vals, const int32_t* __restrict__ done) {
    constexpr int S = 1 << L0;
    constexpr int S2 = S * S, S3 = S * S * S;
    __shared__ double nA[kCubeLds / 4];
    __shared__ double nB[kCubeLds / 4];
    __shared__ double P[kCubeLds];
    if (done && *done) return;
    int64_t ncubes = *ncubes_p;
    if (ncubes > cap) ncubes = cap;
    const double t0 = (MODE == 1 && tau0_p) ? *tau0_p : 0.0;
    const int tid = threadIdx.x;
    for (int64_t g = blockIdx.x; g * cpw < ncubes; g += gridDim.x) {
        const int64_t c0 = g * cpw;
        __syncthreads();
        for (int t = tid; t < cpw * S2; t += 256) {
            const int c = t / S2, r = t % S2;
            const int a = r / S, q = r % S;
            double va = 0.0, vb = 0.0;
            if (c0 + c < ncubes) {
                uint32_t I, K, J;
                demorton3(keys[c0 + c], I, K, J);
                const int i = (int)I * S + a, k = (int)K * S + q;  // A_ik
                if (i < nb && k < nb) {
                    const int sa = mapA[(size_t)i * nb + k];
                    if (sa >= 0) va = normA[sa];
                }
                const int kk = (int)K * S + a, j = (int)J * S + q;  // B_kj
                if (kk < nb && j < nb) {
                    const int sb = btrans ? mapB[(size_t)j * nb + kk] : mapB[(size_t)kk * nb + j];
                    if (sb >= 0) vb = normB[sb];
                }
            }
            nA[t] = va;
            nB[t] = vb;
        }
        __syncthreads();
        for (int t = tid; t < cpw * S3; t += 256) {
            const int c = t / S3, r = t % S3;
            const int i = r / S2, k = (r / S) % S, j = r % S;
            P[t] = nA[c * S2 + i * S + k] * nB[c * S2 + k * S + j];
        }
        __syncthreads();
        const int c = tid / lpc;
        if (c < cpw && c0 + c < ncubes) {
            for (int m = tid % lpc; m < N; m += lpc)
                vals[(size_t)(c0 + c) * N + m] = cube_node<L0, S, MODE>(0, 0, 0, tau[m], t0, c_low, P + c * S3);
        }
    }
}

// More candidates: each workgroup of 256 threads takes one cube and
// kCandPerWg candidates:
// the cube's A and B leaf norms go to LDS, then its S^3 leaf products
// (computed once per workgroup, shared by its candidates); eight threads per
// candidate evaluate the cube's eight level-(L0 - 1) subtrees (octant
// q = a kappa c, Algorithm 3's order inside each), and the first of the
// eight combines them as the root of the subtree does: a outer, c inner,
// t = E(a, 0, c) + E(a, 1, c), acc += t^2, then the root.  The same
// operations as one thread walking the whole cube, so the values are the
// same; the eight shorter dependence chains keep more of the CU busy.
constexpr int kCandPerWg = 256 / 8;

template <int L0, int MODE>
__global__ __launch_bounds__(256) void k_cube_eval_split(int nb, const uint32_t* __restrict__ keys,
                                                  const int64_t* __restrict__ ncubes_p, int64_t cap,
                                                  const int32_t* __restrict__ mapA, const double* __restrict__ normA,
                                                  const int32_t* __restrict__ mapB, const double* __restrict__ normB,
                                                  int btrans, const double* __restrict__ tau, int N,
                                                  const double* __restrict__ tau0_p, double c_low, int slices,
                                                  double* __restrict__ vals, const int32_t* __restrict__ done) {
    constexpr int S = 1 << L0;
    constexpr int S2 = S * S, S3 = S * S * S;
    __shared__ double nA[S2];
    __shared__ double nB[S2];
    __shared__ double P[S3];
    if (done && *done) return;
    int64_t ncubes = *ncubes_p;
    if (ncubes > cap) ncubes = cap;
    const double t0 = (MODE == 1 && tau0_p) ? *tau0_p : 0.0;
    const int tid = threadIdx.x, lane = tid & 63;
    const int q = tid & 7;
    for (int64_t g = blockIdx.x; g < ncubes * slices; g += gridDim.x) {
        const int64_t cube = g / slices;
        const int m = (int)(g - cube * slices) * kCandPerWg + (tid >> 3);
        __syncthreads();
        uint32_t I, K, J;
        demorton3(keys[cube], I, K, J);
        for (int t = tid; t < S2; t += 256) {
            const int a = t / S, r = t % S;
            double va = 0.0, vb = 0.0;
            const int i = (int)I * S + a, k = (int)K * S + r;  // A_ik
            if (i < nb && k < nb) {
                const int sa = mapA[(size_t)i * nb + k];
                if (sa >= 0) va = normA[sa];
            }
            const int kk = (int)K * S + a, j = (int)J * S + r;  // B_kj
            if (kk < nb && j < nb) {
                const int sb = btrans ? mapB[(size_t)j * nb + kk] : mapB[(size_t)kk * nb + j];
                if (sb >= 0) vb = normB[sb];
            }
            nA[t] = va;
            nB[t] = vb;
        }
        __syncthreads();
        for (int t = tid; t < S3; t += 256) {
            const int i = t / S2, k = (t / S) % S, j = t % S;
            P[t] = nA[i * S + k] * nB[k * S + j];
        }
        __syncthreads();
        double e = 0.0;
        if constexpr (L0 == 0) {
            if (m < N && q == 0) e = cube_node<0, S, MODE>(0, 0, 0, tau[m], t0, c_low, P);
        } else {
            if (m < N) e = cube_node<L0 - 1, S, MODE>(q >> 2, (q >> 1) & 1, q & 1, tau[m], t0, c_low, P);
        }
        double ev[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) ev[u] = __shfl(e, (lane & ~7) | u);
        if (q == 0 && m < N) {
            double v = ev[0];
            if constexpr (L0 > 0) {
                double acc = 0.0;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        double t = ev[(a << 2) | c] + ev[(a << 2) | 2 | c];
                        double t2 = t * t;
                        acc = acc + t2;
                    }
                v = sqrt(acc);
            }
            vals[(size_t)cube * N + m] = v;
        }
    }
}

// kernel<L0, MODE> for the runtime l0 (0..4) and mode (0, 1)
template <template <int, int> class K, typename... Args>
void launch_cube_kernel(int mode, int l0, dim3 grid, hipStream_t s, Args... args) {
#define SPAMM_CUBE(L0_, M_) hipLaunchKernelGGL((K<L0_, M_>::fn), grid, dim3(256), 0, s, args...)
    if (mode == 0) {
        switch (l0) {
            case 0: SPAMM_CUBE(0, 0); break;
            case 1: SPAMM_CUBE(1, 0); break;
            case 2: SPAMM_CUBE(2, 0); break;
            case 3: SPAMM_CUBE(3, 0); break;
            case 4: SPAMM_CUBE(4, 0); break;
        }
    } else {
        switch (l0) {
            case 0: SPAMM_CUBE(0, 1); break;
            case 1: SPAMM_CUBE(1, 1); break;
            case 2: SPAMM_CUBE(2, 1); break;
            case 3: SPAMM_CUBE(3, 1); break;
            case 4: SPAMM_CUBE(4, 1); break;
        }
    }
#undef SPAMM_CUBE
}
template <int L0, int MODE>
struct CubeWhole {
    static constexpr auto fn = k_cube_eval_whole<L0, MODE>;
};
template <int L0, int MODE>
struct CubeSplit {
    static constexpr auto fn = k_cube_eval_split<L0, MODE>;
};

void launch_cube_eval(int mode, int l0, int nb, const uint32_t* keys, const int64_t* ncubes, int64_t cap,
                      const int32_t* mapA, const double* normA, const int32_t* mapB, const double* normB, int btrans,
                      const double* tau, int N, const double* tau0, double c_low, double* vals, const int32_t* done,
                      hipStream_t s) {
    if (N <= 64) {
        // threads per cube: the candidate count rounded up to a power of two,
        // cubes per workgroup: what 256 threads and the LDS hold
        int lpc = 1;
        while (lpc < N) lpc <<= 1;
        const int s3 = 1 << (3 * l0);
        int cpw = 256 / lpc;
        while (cpw > 1 && cpw * s3 > kCubeLds) cpw >>= 1;
        const int grid = grid_for((cap + cpw - 1) / cpw, 1, 4096);
        launch_cube_kernel<CubeWhole>(mode, l0, dim3(grid), s, nb, keys, ncubes, cap, mapA, normA, mapB, normB,
                                      btrans, tau, N, tau0, c_low, cpw, lpc, vals, done);
        return;
    }
    const int slices = (N + kCandPerWg - 1) / kCandPerWg;
    const int grid = grid_for(cap * slices, 1, 8192);
    launch_cube_kernel<CubeSplit>(mode, l0, dim3(grid), s, nb, keys, ncubes, cap, mapA, normA, mapB, normB, btrans,
                                  tau, N, tau0, c_low, slices, vals, done);
}

__global__ void k_level_flags(const uint32_t* __restrict__ keys, const int64_t* __restrict__ n_p, int64_t cap,
                              int32_t* __restrict__ flag, const int32_t* __restrict__ done) {
    if (done && *done) return;
    int64_t n = *n_p;
    if (n > cap) n = cap;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        flag[c] = (c == 0 || (keys[c] >> 3) != (keys[c - 1] >> 3)) ? 1 : 0;
}

void launch_level_flags(const uint32_t* keys, const int64_t* n, int64_t cap, int32_t* flag, const int32_t* done,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_level_flags, dim3(grid_for(cap, 256, 4096)), dim3(256), 0, s, keys, n, cap, flag, done);
}

__global__ void k_level_build(const uint32_t* __restrict__ keys, const int64_t* __restrict__ n_p, int64_t cap,
                              const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                              const int64_t* __restrict__ np_p, uint32_t* __restrict__ pkeys,
                              int32_t* __restrict__ pstart, const int32_t* __restrict__ done) {
    if (done && *done) return;
    int64_t n = *n_p;
    if (n > cap) n = cap;
    if (blockIdx.x == 0 && threadIdx.x == 0) pstart[*np_p] = (int32_t)n;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        if (flag[c]) {
            int p = pos[c];
            pkeys[p] = keys[c] >> 3;
            pstart[p] = (int32_t)c;
        }
    }
}

void launch_level_build(const uint32_t* keys, const int64_t* n, int64_t cap, const int32_t* flag, const int32_t* pos,
                        const int64_t* nparent, uint32_t* pkeys, int32_t* pstart, const int32_t* done, hipStream_t s) {
    hipLaunchKernelGGL(k_level_build, dim3(grid_for(cap, 256, 4096)), dim3(256), 0, s, keys, n, cap, flag, pos,
                       nparent, pkeys, pstart, done);
}

// Error value of one octree node for candidate m from its present children
// c0 .. c1 - 1 (octant = key & 7, absent children count as zero): the
// combination of Algorithm 3, a (row half of C) outer, c (column half)
// inner, t = E(a, k=0, c) + E(a, k=1, c), acc += t^2, then the root.
SPAMM_DEV double node_eval(const uint32_t* ckeys, const double* __restrict__ cvals, int c0, int c1, int m, int N) {
    // a node has at most eight children: all their loads issued before any is used
    uint32_t o[8];
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const bool live = c0 + u < c1;
        o[u] = live ? (ckeys[c0 + u] & 7u) : 8u;
        v[u] = live ? cvals[(size_t)(c0 + u) * N + m] : 0.0;
    }
    double e[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) e[q] = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int q = 0; q < 8; ++q) e[q] = (o[u] == (uint32_t)q) ? v[u] : e[q];
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            double t = e[(a << 2) | c] + e[(a << 2) | 2 | c];
            double t2 = t * t;
            acc = acc + t2;
        }
    return sqrt(acc);
}

__global__ void k_level_eval(const uint32_t* __restrict__ ckeys, const double* __restrict__ cvals,
                             const int32_t* __restrict__ pstart, const int64_t* __restrict__ np_p, int64_t cap, int N,
                             double* __restrict__ pvals, const int32_t* __restrict__ done) {
    if (done && *done) return;
    int64_t np = *np_p;
    if (np > cap) np = cap;
    const int64_t total = np * N;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = idx / N;
        const int m = (int)(idx - p * N);
        pvals[(size_t)p * N + m] = node_eval(ckeys, cvals, pstart[p], pstart[p + 1], m, N);
    }
}

// The top levels of the octree in one workgroup: from the n <= kTopNodes
// sorted nodes of one level (keys_in, values va) up to the root, level by
// level exactly as k_level_flags / scan / build / eval do, with the node
// lists in LDS and the values alternating between va and vb; then the
// selection (as k_select).  Replaces six launches per level and the
// selection's launch.
constexpr int kTopThreads = 1024;
__global__ __launch_bounds__(kTopThreads) void k_levels_top(const uint32_t* __restrict__ keys_in,
                                                          const int64_t* __restrict__ n_in, double* va, double* vb,
                                                          int nlev, int N, const double* __restrict__ tau,
                                                          const double* __restrict__ budget_dev, double budget_host,
                                                          double* __restrict__ bound_out,
                                                          int32_t* __restrict__ idx_out, double* __restrict__ tau_out,
                                                          const int32_t* __restrict__ done) {
    __shared__ uint32_t keys[2][kTopNodes];
    __shared__ int32_t pstart[kTopNodes + 1];
    __shared__ int32_t wsum[kTopThreads / 64];
    __shared__ int best;
    if (done && *done) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int n = (int)(*n_in < (int64_t)kTopNodes ? *n_in : (int64_t)kTopNodes);
    for (int c = tid; c < n; c += kTopThreads) keys[0][c] = keys_in[c];
    __syncthreads();
    int cur = 0;
    const double* cv = va;
    double* pv = vb;
    for (int lev = 0; lev < nlev; ++lev) {
        // parents: the first child of each run of equal key >> 3 starts a parent
        int np = 0;
        for (int c0 = 0; c0 < n; c0 += kTopThreads) {
            const int c = c0 + tid;
            const bool f = c < n && (c == 0 || (keys[cur][c] >> 3) != (keys[cur][c - 1] >> 3));
            const uint64_t bal = __ballot(f);
            if (lane == 0) wsum[w] = __popcll(bal);
            __syncthreads();
            int off = np, tot = 0;
            for (int q = 0; q < kTopThreads / 64; ++q) {
                if (q < w) off += wsum[q];
                tot += wsum[q];
            }
            if (f) {
                const int pos = off + __popcll(bal & ((1ull << lane) - 1ull));
                keys[1 - cur][pos] = keys[cur][c] >> 3;
                pstart[pos] = c;
            }
            np += tot;
            __syncthreads();
        }
        if (tid == 0) pstart[np] = n;
        __syncthreads();
        // four nodes per thread and round, their child loads all issued
        // before the first result is stored (the stores may alias the
        // children's values as far as the compiler knows)
        constexpr int U = 4;
        const int tot = np * N;
        for (int idx0 = tid; idx0 < tot; idx0 += U * kTopThreads) {
            double r[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = idx0 + u * kTopThreads;
                if (idx < tot) {
                    const int p = idx / N, m = idx - p * N;
                    r[u] = node_eval(keys[cur], cv, pstart[p], pstart[p + 1], m, N);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = idx0 + u * kTopThreads;
                if (idx < tot) pv[idx] = r[u];  // idx = p N + m
            }
        }
        __syncthreads();
        cur = 1 - cur;
        n = np;
        const double* t = cv;
        cv = pv;
        pv = const_cast<double*>(t);
    }
    // selection: the first (largest) candidate whose bound is below the budget
    if (tid == 0) best = N;
    __syncthreads();
    const double budget = budget_dev ? *budget_dev : budget_host;
    for (int m = tid; m < N; m += kTopThreads) {
        const double bd = n > 0 ? cv[m] : 0.0;
        if (bound_out) bound_out[m] = bd;
        if (bd < budget) atomicMin(&best, m);
    }
    __syncthreads();
    if (tid == 0) {
        *idx_out = best;
        *tau_out = best < N ? tau[best] : 0.0;
    }
}

void launch_levels_top(const uint32_t* keys, const int64_t* n, double* va, double* vb, int nlev, int N,
                       const double* tau, const double* budget_dev, double budget_host, double* bound_out,
                       int32_t* idx_out, double* tau_out, const int32_t* done, hipStream_t s) {
    hipLaunchKernelGGL(k_levels_top, dim3(1), dim3(kTopThreads), 0, s, keys, n, va, vb, nlev, N, tau, budget_dev,
                       budget_host, bound_out, idx_out, tau_out, done);
}

void launch_level_eval(const uint32_t* ckeys, const double* cvals, const int32_t* pstart, const int64_t* nparent,
                       int64_t cap, int N, double* pvals, const int32_t* done, hipStream_t s) {
    hipLaunchKernelGGL(k_level_eval, dim3(grid_for(cap * N, 256, 8192)), dim3(256), 0, s, ckeys, cvals, pstart, nparent,
                       cap, N, pvals, done);
}

// Selection: the first (largest) candidate whose bound is below the budget;
// none -> index N and tau = 0 (exact product).
__global__ __launch_bounds__(1024) void k_select(const double* __restrict__ root, const int64_t* __restrict__ nroot,
                                                const double* __restrict__ tau, int N,
                                                const double* __restrict__ budget_dev, double budget_host,
                                                double* __restrict__ bound_out, int32_t* __restrict__ idx_out,
                                                double* __restrict__ tau_out, const int32_t* __restrict__ done) {
    __shared__ int best;
    if (done && *done) return;
    if (threadIdx.x == 0) best = N;
    __syncthreads();
    const double budget = budget_dev ? *budget_dev : budget_host;
    const bool have = *nroot > 0;
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        double bd = have ? root[m] : 0.0;
        if (bound_out) bound_out[m] = bd;
        if (bd < budget) atomicMin(&best, m);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        *idx_out = best;
        *tau_out = best < N ? tau[best] : 0.0;
    }
}

void launch_select(const double* root, const int64_t* nroot, const double* tau, int N, const double* budget_dev,
                   double budget_host, double* bound_out, int32_t* idx_out, double* tau_out, const int32_t* done,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, root, nroot, tau, N, budget_dev, budget_host, bound_out,
                       idx_out, tau_out, done);
}

}  // namespace spamm
