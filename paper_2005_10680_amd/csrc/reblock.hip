// Re-blocking: the same n x n matrix on another leaf size (b -> 2b merges
// 2 x 2 block quads, 2b -> b splits blocks).  A block of the new grid is
// present when any block of the old grid it overlaps is present
// (structural; split-off all-zero blocks stay present with zero values and
// norm 0, so they are skipped by any tau > 0 and removed by the first
// truncation).  Slots of the result are assigned in 2D Morton order of the
// new grid, like every matrix the library produces.
#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

SPAMM_DEV bool overlaps_present(const MatView& X, int R, int C, int b2) {
    const int b = X.b, nb = X.nb;
    const int r0 = (int)(((int64_t)R * b2) / b), r1 = (int)(((int64_t)(R + 1) * b2 - 1) / b);
    const int c0 = (int)(((int64_t)C * b2) / b), c1 = (int)(((int64_t)(C + 1) * b2 - 1) / b);
    for (int r = r0; r <= r1 && r < nb; ++r)
        for (int c = c0; c <= c1 && c < nb; ++c)
            if (X.map[(size_t)r * nb + c] >= 0) return true;
    return false;
}

__global__ void k_reblock_flags(MatView X, int b2, int nb2, int P, int32_t* __restrict__ flag) {
    const int64_t PP = (int64_t)P * P;
    for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < PP; z += (int64_t)gridDim.x * blockDim.x) {
        uint32_t R, C;
        demorton2((uint32_t)z, R, C);
        flag[z] = ((int)R < nb2 && (int)C < nb2 && overlaps_present(X, (int)R, (int)C, b2)) ? 1 : 0;
    }
}

__global__ void k_reblock_assign(int nb2, int P, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                                 const int64_t* __restrict__ total, MatView Y, int32_t* __restrict__ ovf) {
    const int64_t PP = (int64_t)P * P;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t t = *total;
        *Y.nslot = (int32_t)(t <= Y.cap ? t : Y.cap);
        if (t > Y.cap) *ovf = 1;
    }
    for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < PP; z += (int64_t)gridDim.x * blockDim.x) {
        uint32_t R, C;
        demorton2((uint32_t)z, R, C);
        if ((int)R >= nb2 || (int)C >= nb2) continue;
        int32_t m = -1;
        if (flag[z]) {
            const int64_t sl = pos[z];
            if (sl < Y.cap) {
                m = (int32_t)sl;
                Y.brow[sl] = (int32_t)R;
                Y.bcol[sl] = (int32_t)C;
            }
        }
        Y.map[(size_t)R * nb2 + C] = m;
    }
}

// one workgroup per slot of Y: every entry from the old grid (0 where the
// old block is absent or past n)
__global__ __launch_bounds__(256) void k_reblock_values(MatView X, MatView Y) {
    int64_t ns = *Y.nslot;
    if (ns > Y.cap) ns = Y.cap;
    const int b = X.b, b2 = Y.b, nb = X.nb;
    const int64_t n = X.n;
    for (int64_t s = blockIdx.x; s < ns; s += gridDim.x) {
        const int R = Y.brow[s], C = Y.bcol[s];
        double* out = Y.val + (size_t)s * b2 * b2;
        for (int e = threadIdx.x; e < b2 * b2; e += 256) {
            const int col = e / b2, row = e % b2;  // column-major inside the block
            const int64_t gr = (int64_t)R * b2 + row, gc = (int64_t)C * b2 + col;
            double v = 0.0;
            if (gr < n && gc < n) {
                const int r = (int)(gr / b), c = (int)(gc / b);
                if (r < nb && c < nb) {
                    const int m = X.map[(size_t)r * nb + c];
                    if (m >= 0) v = X.val[(size_t)m * b * b + (size_t)(gc % b) * b + (gr % b)];
                }
            }
            out[e] = v;
        }
    }
}

void launch_reblock(const MatView& X, const MatView& Y, int32_t* flag, int32_t* pos, int64_t* total, void* scan_tmp,
                    int32_t* ovf, hipStream_t s) {
    int P = 1;
    while (P < Y.nb) P <<= 1;
    const int64_t PP = (int64_t)P * P;
    hipLaunchKernelGGL(k_reblock_flags, dim3(grid_for(PP, 256, 8192)), dim3(256), 0, s, X, Y.b, Y.nb, P, flag);
    scan_i32(flag, pos, PP, nullptr, total, scan_tmp, s);
    hipLaunchKernelGGL(k_reblock_assign, dim3(grid_for(PP, 256, 8192)), dim3(256), 0, s, Y.nb, P, flag, pos, total, Y,
                       ovf);
    hipLaunchKernelGGL(k_reblock_values, dim3(grid_for(Y.cap, 1, 16384)), dim3(256), 0, s, X, Y);
}

}  // namespace spamm
