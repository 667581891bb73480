// Leaf-level error bounds over the skipped block pairs (alternatives to the
// recursive bound of Algorithm 3, computed for every candidate threshold):
//   sum : B_sum(tau)  = sum over all skipped triples (i,k,j) of p_ikj,
//   flat: B_flat(tau) = sqrt(sum over outputs (i,j) of (sum_{k skipped} p_ikj)^2),
// p_ikj = RN(nu(A_ik) nu(B_kj)), skipped iff p < tau.  B_flat is eq. (6)
// applied at the leaves: ||E_ij||_F <= sum_k ||A_ik||_F ||B_kj||_F for the
// skipped k of each output block, so ||E||_F <= B_flat <= B_tree (Algorithm
// 3's bound) <= B_sum.
//
// One wave per output block.  The wave first gathers the output's present
// products p_ikj in ascending k into its LDS row (64 inner indices at a
// time: each lane tests one k, the lanes' loads are independent, and a
// ballot compacts the present ones), then lane m (and m + 64, ...) adds
// the p below its own threshold tau_m along that row: per output and
// candidate the same k-ascending sum the oracle forms.  Per-wave partial
// sums over outputs go to a partial array and a second kernel adds the
// partials in a fixed order, so the results are deterministic.
#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

template <int R>
__global__ __launch_bounds__(256) void k_bound_part(int nb, int nw, const uint32_t* __restrict__ bitsA,
                                                   const uint32_t* __restrict__ bitsB,
                                                   const int32_t* __restrict__ mapA, const double* __restrict__ normA,
                                                   const int32_t* __restrict__ mapB, const double* __restrict__ normB,
                                                   int btrans, const double* __restrict__ tau, int N, int flat,
                                                   int mode, const double* __restrict__ tau0_p, double c_low,
                                                   double* __restrict__ part, const int32_t* __restrict__ done) {
    extern __shared__ double prow[];  // [4][nb]
    if (done && *done) return;
    const double t0 = (mode == 1 && tau0_p) ? *tau0_p : 0.0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double* row = prow + (size_t)w * nb;
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
        for (int r = 0; r < R; ++r) acc[r] = acc[r] + (flat ? s[r] * s[r] : s[r]);
        // the row is rewritten by the next output: every lane must be done reading
        __builtin_amdgcn_wave_barrier();
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

// the LDS rows limit the leaf-level bounds to nb <= kBoundMaxNb (64 KB per workgroup)
int64_t bound_part_waves(int nb) {
    const int64_t nout = (int64_t)nb * nb;
    int64_t blocks = (nout + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    return blocks * 4;
}

void launch_bound_leaf(int nb, int nw, const uint32_t* bitsA, const uint32_t* bitsB, const int32_t* mapA,
                       const double* normA, const int32_t* mapB, const double* normB, int btrans, const double* tau,
                       int N, int flat, int mode, const double* tau0, double c_low, double* part, double* out,
                       const int32_t* done, hipStream_t s) {
    const int64_t nw_waves = bound_part_waves(nb);
    const int grid = (int)(nw_waves / 4);
    const size_t lds = sizeof(double) * 4 * (size_t)nb;  // one row of nb products per wave
#define SPAMM_BP(R_)                                                                                             \
    hipLaunchKernelGGL((k_bound_part<R_>), dim3(grid), dim3(256), lds, s, nb, nw, bitsA, bitsB, mapA, normA, mapB, \
                       normB, btrans, tau, N, flat, mode, tau0, c_low, part, done)
    if (N <= 64) SPAMM_BP(1);
    else if (N <= 128) SPAMM_BP(2);
    else if (N <= 256) SPAMM_BP(4);
    else if (N <= 512) SPAMM_BP(8);
    else SPAMM_BP(16);
#undef SPAMM_BP
    hipLaunchKernelGGL(k_bound_final, dim3(N), dim3(256), 0, s, part, nw_waves, N, flat, out, done);
}

}  // namespace spamm
