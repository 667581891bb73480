// Leaf-level error bounds over the skipped block pairs (alternatives to the
// recursive bound of Algorithm 3, computed for every candidate threshold):
//   sum : B_sum(tau)  = sum over all skipped triples (i,k,j) of p_ikj,
//   flat: B_flat(tau) = sqrt(sum over outputs (i,j) of (sum_{k skipped} p_ikj)^2),
// p_ikj = RN(nu(A_ik) nu(B_kj)), skipped iff p < tau.  B_flat is eq. (6)
// applied at the leaves: ||E_ij||_F <= sum_k ||A_ik||_F ||B_kj||_F for the
// skipped k of each output block, so ||E||_F <= B_flat <= B_tree (Algorithm
// 3's bound) <= B_sum.
//
// One wave per output block, one lane per candidate (lane m, m + 64, ...):
// every lane walks the output's present pairs in ascending k and adds the p
// below its own threshold, so each lane holds the prefix of the output's
// sorted products below tau_m without sorting them.  Per-wave partial sums
// go to a partial array and a second kernel adds the partials in a fixed
// order, so the results are deterministic.
#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

template <int R>
__global__ __launch_bounds__(256) void k_bound_part(int nb, int nw, const uint32_t* __restrict__ bitsA,
                                                   const uint32_t* __restrict__ bitsB,
                                                   const int32_t* __restrict__ mapA, const double* __restrict__ normA,
                                                   const int32_t* __restrict__ mapB, const double* __restrict__ normB,
                                                   int btrans, const double* __restrict__ tau, int N, int flat,
                                                   double* __restrict__ part, const int32_t* __restrict__ done) {
    if (done && *done) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double tm[R], acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int m = lane + 64 * r;
        tm[r] = m < N ? tau[m] : 0.0;
        acc[r] = 0.0;
    }
    const int64_t nout = (int64_t)nb * nb;
    const int64_t wid = (int64_t)blockIdx.x * 4 + w, nwaves = (int64_t)gridDim.x * 4;
    for (int64_t z = wid; z < nout; z += nwaves) {
        const int i = (int)(z / nb), j = (int)(z % nb);
        double s[R];
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] = 0.0;
        for_each_kept(i, j, nb, nw, bitsA, bitsB, mapA, normA, mapB, normB, btrans, 0.0,
                      [&](int, int, int, double p) {
#pragma unroll
                          for (int r = 0; r < R; ++r) s[r] = (p < tm[r]) ? s[r] + p : s[r];
                      });
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = acc[r] + (flat ? s[r] * s[r] : s[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int m = lane + 64 * r;
        if (m < N) part[(size_t)wid * N + m] = acc[r];
    }
}

// One workgroup per candidate: thread t adds partials t, t + 256, ... in
// order, then a fixed-shape tree adds the 256 thread sums.
__global__ __launch_bounds__(256) void k_bound_final(const double* __restrict__ part, int64_t nparts, int N, int flat,
                                                    double* __restrict__ out, const int32_t* __restrict__ done) {
    __shared__ double red[256];
    if (done && *done) return;
    const int m = blockIdx.x;
    double t = 0.0;
    for (int64_t q = threadIdx.x; q < nparts; q += 256) t = t + part[(size_t)q * N + m];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[m] = flat ? sqrt(red[0]) : red[0];
}

int64_t bound_part_waves(int nb) {
    const int64_t nout = (int64_t)nb * nb;
    int64_t blocks = (nout + 3) / 4;
    if (blocks > 1024) blocks = 1024;
    return blocks * 4;
}

void launch_bound_leaf(int nb, int nw, const uint32_t* bitsA, const uint32_t* bitsB, const int32_t* mapA,
                       const double* normA, const int32_t* mapB, const double* normB, int btrans, const double* tau,
                       int N, int flat, double* part, double* out, const int32_t* done, hipStream_t s) {
    const int64_t nw_waves = bound_part_waves(nb);
    const int grid = (int)(nw_waves / 4);
#define SPAMM_BP(R_)                                                                                             \
    hipLaunchKernelGGL((k_bound_part<R_>), dim3(grid), dim3(256), 0, s, nb, nw, bitsA, bitsB, mapA, normA, mapB, \
                       normB, btrans, tau, N, flat, part, done)
    if (N <= 64) SPAMM_BP(1);
    else if (N <= 128) SPAMM_BP(2);
    else if (N <= 256) SPAMM_BP(4);
    else if (N <= 512) SPAMM_BP(8);
    else SPAMM_BP(16);
#undef SPAMM_BP
    hipLaunchKernelGGL(k_bound_final, dim3(N), dim3(256), 0, s, part, nw_waves, N, flat, out, done);
}

}  // namespace spamm
