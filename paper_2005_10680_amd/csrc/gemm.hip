// K3: leaf products of the kept pairs (the "lowest level" of Algorithm 2),
// FP64 on the CDNA matrix cores.
//
// One workgroup (4 waves) owns one output block C_ij = sum_k A_ik B_kj and
// walks its kept pairs in ascending k.  The inner dimension of all pairs is
// streamed in chunks of KC: the A chunk (KC columns of the column-major A_ik)
// and the B chunk (KC rows of B_kj) are staged through a double-buffered LDS
// tile while the next chunk is in flight.  Each wave accumulates a
// (B/2) x (B/2) quadrant with V_MFMA_F64_16X16X4_F64.  The SP2 combine
// (X^ = C or 2X - C) is fused into the epilogue, and in symmetric mode the
// mirrored block C_ji = C_ij^T is written from the same registers.
//
// The kernel is persistent: the grid is a multiple of the 8 XCDs, the output
// list (Morton order) is cut into 8 contiguous ranges of equal kept-pair
// count, and the workgroups of XCD x take outputs of range x from an atomic
// counter, so neighbouring outputs -- which share A rows and B columns --
// run under the same L2.  Every output is computed by exactly one workgroup
// in a fixed order: results are bitwise reproducible.
#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int B>
struct GemmCfg {
    static constexpr int TM = B / 32;  // 16x16 tiles per wave along rows (2 waves)
    static constexpr int TN = B / 32;  // along columns (2 waves)
    static constexpr int KC = 16;      // inner indices per LDS stage
    static constexpr int CH = B / KC;  // stages per kept pair
    static constexpr int LD = B + 4;   // LDS row stride (doubles)
    static constexpr int V2PT = KC * B / 2 / 256;  // double2 loads per thread per operand
};

// Staging registers as one vector value (kept in VGPRs, never in scratch).
template <int N>
struct DVec {
    typedef double type __attribute__((ext_vector_type(N)));
};
template <int B>
using StageV = typename DVec<2 * GemmCfg<B>::V2PT>::type;

// Global -> register stage of one chunk: the A chunk is KC contiguous columns
// of A_ik; the B chunk is KC contiguous columns of Bt_jk (BT) or KC rows of
// the column-major B_kj.
template <int B, bool BT>
SPAMM_DEV void load_stage(StageV<B>& sa, StageV<B>& sb, const double* __restrict__ valA, const double* __restrict__ valB, int2 pr, int chunk) {
    using C = GemmCfg<B>;
    const int t = threadIdx.x;
    const double* a0 = valA + (size_t)pr.x * B * B + (size_t)chunk * C::KC * B;
#pragma unroll
    for (int v = 0; v < C::V2PT; ++v) {
        const double2 x = reinterpret_cast<const double2*>(a0)[t + 256 * v];
        sa[2 * v] = x.x;
        sa[2 * v + 1] = x.y;
    }
    if constexpr (BT) {
        const double* b0 = valB + (size_t)pr.y * B * B + (size_t)chunk * C::KC * B;
#pragma unroll
        for (int v = 0; v < C::V2PT; ++v) {
            const double2 x = reinterpret_cast<const double2*>(b0)[t + 256 * v];
            sb[2 * v] = x.x;
            sb[2 * v + 1] = x.y;
        }
    } else {
        const double* b0 = valB + (size_t)pr.y * B * B + (size_t)chunk * C::KC;
#pragma unroll
        for (int v = 0; v < C::V2PT; ++v) {
            const int idx = t + 256 * v;
            const int col = idx / (C::KC / 2), kp = idx % (C::KC / 2);
            const double2 x = *reinterpret_cast<const double2*>(b0 + (size_t)col * B + 2 * kp);
            sb[2 * v] = x.x;
            sb[2 * v + 1] = x.y;
        }
    }
}

// Register -> LDS: both tiles are stored [k][row or column].
template <int B, bool BT>
SPAMM_DEV void store_stage(const StageV<B>& sa, const StageV<B>& sb, double* As, double* Bs) {
    using C = GemmCfg<B>;
    const int t = threadIdx.x;
#pragma unroll
    for (int v = 0; v < C::V2PT; ++v) {
        const int e = 2 * (t + 256 * v);
        const int k = e / B, r = e % B;
        *reinterpret_cast<double2*>(As + k * C::LD + r) = double2{sa[2 * v], sa[2 * v + 1]};
    }
    if constexpr (BT) {
#pragma unroll
        for (int v = 0; v < C::V2PT; ++v) {
            const int e = 2 * (t + 256 * v);
            const int k = e / B, c = e % B;
            *reinterpret_cast<double2*>(Bs + k * C::LD + c) = double2{sb[2 * v], sb[2 * v + 1]};
        }
    } else {
#pragma unroll
        for (int v = 0; v < C::V2PT; ++v) {
            const int idx = t + 256 * v;
            const int col = idx / (C::KC / 2), kp = idx % (C::KC / 2);
            Bs[(2 * kp) * C::LD + col] = sb[2 * v];
            Bs[(2 * kp + 1) * C::LD + col] = sb[2 * v + 1];
        }
    }
}

template <int B, bool BT>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs g) {
    using C = GemmCfg<B>;
    __shared__ __attribute__((aligned(16))) double lds[2][2][C::KC * C::LD];
    __shared__ int s_o, s_lo, s_hi;
    if (g.done && *g.done) return;
    if (g.ovf && *g.ovf) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int64_t nout = *g.nout;
    const int nx = gridDim.x / 8;
    const int xcd = blockIdx.x % 8;
    if (tid == 0) {
        // pair-balanced contiguous range of outputs for this XCD
        const int64_t np = g.optr[nout];
        const int64_t t_lo = np * xcd / 8, t_hi = np * (xcd + 1) / 8;
        int64_t lo = 0, hi = nout;
        while (lo < hi) {  // first o with optr[o] >= t_lo
            int64_t mid = (lo + hi) >> 1;
            if (g.optr[mid] < t_lo) lo = mid + 1; else hi = mid;
        }
        s_lo = (int)lo;
        int64_t l2 = 0, h2 = nout;
        while (l2 < h2) {
            int64_t mid = (l2 + h2) >> 1;
            if (g.optr[mid] < t_hi) l2 = mid + 1; else h2 = mid;
        }
        s_hi = xcd == 7 ? (int)nout : (int)l2;
    }
    __syncthreads();
    const int lo = s_lo, hi = s_hi;
    (void)nx;
    const bool beta = g.mapX && g.branch && (*g.branch == 1);

    while (true) {
        if (tid == 0) s_o = lo + atomicAdd(&g.counters[xcd], 1);
        __syncthreads();
        const int o = s_o;
        __syncthreads();
        if (o >= hi) break;
        const int i = g.oi[o], j = g.oj[o];
        const int p0 = g.optr[o], p1 = g.optr[o + 1];
        const int nch = (p1 - p0) * C::CH;

        d4 acc[C::TM][C::TN];
#pragma unroll
        for (int a = 0; a < C::TM; ++a)
#pragma unroll
            for (int b = 0; b < C::TN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

        StageV<B> sa, sb;
        if (nch > 0) {
            load_stage<B, BT>(sa, sb, g.valA, g.valB, g.pairs[p0], 0);
            store_stage<B, BT>(sa, sb, lds[0][0], lds[0][1]);
        }
        __syncthreads();
        for (int gi = 0; gi < nch; ++gi) {
            const int buf = gi & 1;
            if (gi + 1 < nch) {
                const int gn = gi + 1;
                load_stage<B, BT>(sa, sb, g.valA, g.valB, g.pairs[p0 + gn / C::CH], gn % C::CH);
            }
            const double* As = lds[buf][0];
            const double* Bs = lds[buf][1];
#pragma unroll
            for (int ks = 0; ks < C::KC / 4; ++ks) {
                const int kr = ks * 4 + (lane >> 4);
                double av[C::TM], bv[C::TN];
#pragma unroll
                for (int a = 0; a < C::TM; ++a) av[a] = As[kr * C::LD + wm * C::TM * 16 + a * 16 + (lane & 15)];
#pragma unroll
                for (int b = 0; b < C::TN; ++b) bv[b] = Bs[kr * C::LD + wn * C::TN * 16 + b * 16 + (lane & 15)];
#pragma unroll
                for (int a = 0; a < C::TM; ++a)
#pragma unroll
                    for (int b = 0; b < C::TN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
            }
            if (gi + 1 < nch) store_stage<B, BT>(sa, sb, lds[buf ^ 1][0], lds[buf ^ 1][1]);
            __syncthreads();
        }

        // epilogue: combine and write (plus the mirrored block)
        const int sh = g.map_out[(size_t)i * g.nb + j];
        const int sht = (g.sym && i != j) ? g.map_out[(size_t)j * g.nb + i] : -1;
        const int sx = beta ? g.mapX[(size_t)i * g.nb + j] : -1;
        if (sh >= 0) {
            double* dst = g.val_out + (size_t)sh * B * B;
            double* dstt = sht >= 0 ? g.val_out + (size_t)sht * B * B : nullptr;
            const double* xs = sx >= 0 ? g.valX + (size_t)sx * B * B : nullptr;
            // V_MFMA_F64_16X16X4_F64 result layout: register r of lane l holds
            // row (l >> 4) + 4 r, column l & 15 of the 16x16 tile.
#pragma unroll
            for (int a = 0; a < C::TM; ++a)
#pragma unroll
                for (int b = 0; b < C::TN; ++b) {
                    const int col = wn * C::TN * 16 + b * 16 + (lane & 15);
                    const int rowb = wm * C::TM * 16 + a * 16 + (lane >> 4);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = rowb + 4 * r;
                        double v = acc[a][b][r];
                        if (beta) {
                            const double x = xs ? xs[(size_t)col * B + row] : 0.0;
                            v = 2.0 * x - v;
                        }
                        dst[(size_t)col * B + row] = v;
                        if (dstt) dstt[(size_t)row * B + col] = v;
                    }
                }
        }
    }
}

__global__ void k_reset_counters(int32_t* c) {
    if (threadIdx.x < 16) c[threadIdx.x] = 0;
}

void launch_gemm_f64(const GemmArgs& g, int num_cu, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, g.counters);
    const int per_cu = g.b == 128 ? 2 : 4;
    int grid = num_cu * per_cu;
    grid = (grid + 7) / 8 * 8;
#define SPAMM_G(B_, T_) hipLaunchKernelGGL((k_gemm_f64<B_, T_>), dim3(grid), dim3(256), 0, s, g)
    if (g.btrans) {
        switch (g.b) {
            case 32: SPAMM_G(32, true); break;
            case 64: SPAMM_G(64, true); break;
            case 128: SPAMM_G(128, true); break;
        }
    } else {
        switch (g.b) {
            case 32: SPAMM_G(32, false); break;
            case 64: SPAMM_G(64, false); break;
            case 128: SPAMM_G(128, false); break;
        }
    }
#undef SPAMM_G
}

}  // namespace spamm
