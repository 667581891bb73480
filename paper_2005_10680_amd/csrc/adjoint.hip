// Reverse mode of the purification with frozen decisions (not in the paper).
//
// One SP2 step with its kept set K = {(i,k,j): RN(nu(X_ik) nu(X_kj)) >= tau}
// (Algorithm 2 at the leaves), its branch and its truncation pattern S'
// held fixed is the map X -> mask_{S'}(f(C(X))), C(X)_ij = sum over kept k of
// X_ik X_kj.  For a symmetric gradient G of the step's output (on S'), the
// gradient with respect to X, on the pattern of X, is
//     Xbar_ik = A_ik + (A^T)_ik                     (x^2)
//     Xbar_ik = 2 G_ik - (A_ik + (A^T)_ik)          (2x - x^2)
// with A_ik = sum_{j: (i,k,j) in K} G_ij X_kj^T the first-factor part; the
// second-factor part equals A^T because K, X and G are symmetric.  Written
// out per output block (i, k), i <= k, both parts are sums of block
// products over one inner index j:
//     first kind   G_ij X_jk   for j with X_kj, G_ij present and
//                              RN(nu(X_ik) nu(X_kj)) >= tau,
//     second kind  X_ij G_jk   for j with X_ij, G_kj present and
//                              RN(nu(X_ik) nu(X_ij)) >= tau,
// so one launch of the leaf-product kernel (transposed-B layout) computes
// Xbar with the combine of the second branch fused into its epilogue.  Pairs
// of the second kind carry the one's complement of their first slot, which
// tells the product kernel to take A from the second pool and B from the
// first.  Outputs are the live blocks of X with i <= k in slot order (the
// linearised quadtree); outputs without pairs still get their epilogue
// (0, or 2 G_ik on the second branch).
#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

// G_s = (D_s + D_m^T) / 2 with m the slot of the mirror block.
template <int B>
__global__ __launch_bounds__(256) void k_sym_half(MatView D, const double* __restrict__ dval,
                                                  double* __restrict__ gval) {
    int64_t nslot = *D.nslot;
    if (nslot > D.cap) nslot = D.cap;
    for (int64_t s = blockIdx.x; s < nslot; s += gridDim.x) {
        const int r = D.brow[s];
        if (r < 0) continue;
        const int c = D.bcol[s];
        const int m = D.map[(size_t)c * D.nb + r];
        const double* a = dval + (size_t)s * B * B;
        const double* t = m >= 0 ? dval + (size_t)m * B * B : nullptr;
        double* o = gval + (size_t)s * B * B;
        for (int e = threadIdx.x; e < B * B; e += 256) {
            const int col = e / B, row = e % B;
            const double bt = t ? t[(size_t)row * B + col] : 0.0;
            o[e] = 0.5 * (a[e] + bt);
        }
    }
}

void launch_sym_half(const MatView& D, const double* dval, double* gval, hipStream_t s) {
    const int grid = grid_for(D.cap, 1, 4096);
    switch (D.b) {
        case 32: hipLaunchKernelGGL((k_sym_half<32>), dim3(grid), dim3(256), 0, s, D, dval, gval); break;
        case 64: hipLaunchKernelGGL((k_sym_half<64>), dim3(grid), dim3(256), 0, s, D, dval, gval); break;
        case 128: hipLaunchKernelGGL((k_sym_half<128>), dim3(grid), dim3(256), 0, s, D, dval, gval); break;
    }
}

// flag[s] = 1 for live slots with brow <= bcol (s < cap; 0 past nslot)
__global__ void k_adj_flag(MatView X, int32_t* __restrict__ flag) {
    int64_t nslot = *X.nslot;
    if (nslot > X.cap) nslot = X.cap;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < X.cap; s += (int64_t)gridDim.x * blockDim.x) {
        int f = 0;
        if (s < nslot) {
            const int r = X.brow[s];
            f = (r >= 0 && r <= X.bcol[s]) ? 1 : 0;
        }
        flag[s] = f;
    }
}

__global__ void k_adj_place(MatView X, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                            int32_t* __restrict__ oi, int32_t* __restrict__ oj) {
    int64_t nslot = *X.nslot;
    if (nslot > X.cap) nslot = X.cap;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslot; s += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[s]) continue;
        const int o = pos[s];
        oi[o] = X.brow[s];
        oj[o] = X.bcol[s];
    }
}

// Eight lanes per output, as the forward kept-pair passes: lane g walks the
// contiguous bitmap words [g nw / 8, (g + 1) nw / 8) of both kinds, so the
// lanes hold ascending j ranges in lane order.
constexpr int kAdjG = 8;

// The pairs of output (i, k) in this lane's words: first kind, then second
// kind, each in ascending j; f(kind, slot of the first operand, slot of the
// second operand).
template <typename Fn>
SPAMM_DEV void adj_lane_pairs(int i, int k, int w0, int w1, int nb, int nw, const uint32_t* bitsX,
                              const uint32_t* bitsG, const int32_t* mapX, const double* normX, const int32_t* mapG,
                              double tau, Fn&& f) {
    const int sik = mapX[(size_t)i * nb + k];
    if (sik < 0) return;
    const double nik = normX[sik];
    for (int w = w0; w < w1; ++w) {
        uint32_t m = bitsX[(size_t)k * nw + w] & bitsG[(size_t)i * nw + w];
        while (m) {
            const int j = w * 32 + __ffs(m) - 1;
            m &= m - 1;
            const int skj = mapX[(size_t)k * nb + j];
            const int sij = mapG[(size_t)i * nb + j];
            if (skj < 0 || sij < 0) continue;
            if (nik * normX[skj] >= tau) f(0, sij, skj);
        }
    }
    for (int w = w0; w < w1; ++w) {
        uint32_t m = bitsX[(size_t)i * nw + w] & bitsG[(size_t)k * nw + w];
        while (m) {
            const int j = w * 32 + __ffs(m) - 1;
            m &= m - 1;
            const int sij = mapX[(size_t)i * nb + j];
            const int skj = mapG[(size_t)k * nb + j];
            if (sij < 0 || skj < 0) continue;
            if (nik * normX[sij] >= tau) f(1, sij, skj);
        }
    }
}

__global__ void k_adj_count(const int64_t* __restrict__ nout_p, const int32_t* __restrict__ oi,
                            const int32_t* __restrict__ oj, int nb, int nw, const uint32_t* __restrict__ bitsX,
                            const uint32_t* __restrict__ bitsG, const int32_t* __restrict__ mapX,
                            const double* __restrict__ normX, const int32_t* __restrict__ mapG, double tau,
                            int32_t* __restrict__ cnt) {
    const int64_t nout = *nout_p;
    const int g = threadIdx.x % kAdjG;
    const int w0 = g * nw / kAdjG, w1 = (g + 1) * nw / kAdjG;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kAdjG);
    for (int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kAdjG; o < nout; o += groups) {
        int c = 0;
        adj_lane_pairs(oi[o], oj[o], w0, w1, nb, nw, bitsX, bitsG, mapX, normX, mapG, tau,
                       [&](int, int, int) { ++c; });
#pragma unroll
        for (int d = 1; d < kAdjG; d <<= 1) c += __shfl_xor(c, d, kAdjG);
        if (g == 0) cnt[o] = c;
    }
}

// optr[nout] = total pairs; flag an overflow of the pair list
__global__ void k_adj_fin(const int64_t* __restrict__ nout_p, const int64_t* __restrict__ npairs_p,
                          int32_t* __restrict__ optr, int64_t cap_pairs, int32_t* __restrict__ ovf) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t np = *npairs_p;
        optr[*nout_p] = (int32_t)(np <= cap_pairs ? np : cap_pairs);
        if (np > cap_pairs) *ovf = 1;
    }
}

// the pairs of output o: first kind (ascending j), then second kind
// (ascending j, first slot stored as its one's complement); each lane's
// first position in each part from scans over the group's lanes
__global__ void k_adj_fill(const int64_t* __restrict__ nout_p, const int32_t* __restrict__ oi,
                           const int32_t* __restrict__ oj, int nb, int nw, const uint32_t* __restrict__ bitsX,
                           const uint32_t* __restrict__ bitsG, const int32_t* __restrict__ mapX,
                           const double* __restrict__ normX, const int32_t* __restrict__ mapG, double tau,
                           const int32_t* __restrict__ optr, int64_t cap_pairs, int2* __restrict__ pairs,
                           const int32_t* __restrict__ ovf) {
    if (*ovf) return;
    const int64_t nout = *nout_p;
    const int g = threadIdx.x % kAdjG;
    const int w0 = g * nw / kAdjG, w1 = (g + 1) * nw / kAdjG;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kAdjG);
    for (int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kAdjG; o < nout; o += groups) {
        const int i = oi[o], k = oj[o];
        int c0 = 0, c1 = 0;
        adj_lane_pairs(i, k, w0, w1, nb, nw, bitsX, bitsG, mapX, normX, mapG, tau, [&](int kind, int, int) {
            if (kind == 0) ++c0;
            else ++c1;
        });
        int s0 = c0, s1 = c1;
#pragma unroll
        for (int d = 1; d < kAdjG; d <<= 1) {
            const int u0 = __shfl_up(s0, d, kAdjG), u1 = __shfl_up(s1, d, kAdjG);
            if (g >= d) {
                s0 += u0;
                s1 += u1;
            }
        }
        const int tot0 = __shfl(s0, kAdjG - 1, kAdjG);
        const int64_t base = optr[o];
        int64_t p0 = base + (s0 - c0), p1 = base + tot0 + (s1 - c1);
        if (c0 + c1 == 0) continue;
        adj_lane_pairs(i, k, w0, w1, nb, nw, bitsX, bitsG, mapX, normX, mapG, tau, [&](int kind, int a, int b) {
            const int64_t p = kind == 0 ? p0 : p1;
            if (p < cap_pairs) pairs[p] = kind == 0 ? make_int2(a, b) : make_int2(~a, b);
            if (kind == 0) ++p0;
            else ++p1;
        });
    }
}

void launch_adj_outputs(const MatView& X, int32_t* flag, int32_t* pos, int32_t* oi, int32_t* oj, int64_t* nout,
                        void* scan_tmp, hipStream_t s) {
    const int grid = grid_for(X.cap, 256, 4096);
    hipLaunchKernelGGL(k_adj_flag, dim3(grid), dim3(256), 0, s, X, flag);
    scan_i32(flag, pos, X.cap, nullptr, nout, scan_tmp, s);
    hipLaunchKernelGGL(k_adj_place, dim3(grid), dim3(256), 0, s, X, flag, pos, oi, oj);
}

void launch_adj_pairs(int nb, int nw, int64_t cap_out, const int64_t* nout, const int32_t* oi, const int32_t* oj,
                      const uint32_t* bitsX, const uint32_t* bitsG, const int32_t* mapX, const double* normX,
                      const int32_t* mapG, double tau, int32_t* cnt, int32_t* optr, int64_t* npairs,
                      int64_t cap_pairs, int2* pairs, int32_t* ovf, void* scan_tmp, hipStream_t s) {
    const int grid = grid_for(cap_out * kAdjG, 256, 8192);
    hipLaunchKernelGGL(k_adj_count, dim3(grid), dim3(256), 0, s, nout, oi, oj, nb, nw, bitsX, bitsG, mapX, normX,
                       mapG, tau, cnt);
    scan_i32(cnt, optr, cap_out, nout, npairs, scan_tmp, s);
    hipLaunchKernelGGL(k_adj_fin, dim3(1), dim3(64), 0, s, nout, npairs, optr, cap_pairs, ovf);
    hipLaunchKernelGGL(k_adj_fill, dim3(grid), dim3(256), 0, s, nout, oi, oj, nb, nw, bitsX, bitsG, mapX, normX,
                       mapG, tau, optr, cap_pairs, pairs, ovf);
}

// Fbar_s = -G0_m / (lmax - lmin) for F's block s at (r, c), m its slot in
// X~_0 (0 where the first truncation removed it)
template <int B>
__global__ __launch_bounds__(256) void k_adj_fbar(MatView F, const int32_t* __restrict__ map0,
                                                  const double* __restrict__ g0, const double* __restrict__ lam,
                                                  double* __restrict__ fbar) {
    const double W = lam[1] - lam[0];
    int64_t nslot = *F.nslot;
    if (nslot > F.cap) nslot = F.cap;
    for (int64_t s = blockIdx.x; s < nslot; s += gridDim.x) {
        const int r = F.brow[s];
        if (r < 0) continue;
        const int c = F.bcol[s];
        const int m = map0[(size_t)r * F.nb + c];
        double* o = fbar + (size_t)s * B * B;
        const double* g = m >= 0 ? g0 + (size_t)m * B * B : nullptr;
        for (int e = threadIdx.x; e < B * B; e += 256) o[e] = g ? -g[e] / W : 0.0;
    }
}

void launch_adj_fbar(const MatView& F, const int32_t* map0, const double* g0, const double* lam, double* fbar,
                     hipStream_t s) {
    const int grid = grid_for(F.cap, 1, 4096);
    switch (F.b) {
        case 32: hipLaunchKernelGGL((k_adj_fbar<32>), dim3(grid), dim3(256), 0, s, F, map0, g0, lam, fbar); break;
        case 64: hipLaunchKernelGGL((k_adj_fbar<64>), dim3(grid), dim3(256), 0, s, F, map0, g0, lam, fbar); break;
        case 128: hipLaunchKernelGGL((k_adj_fbar<128>), dim3(grid), dim3(256), 0, s, F, map0, g0, lam, fbar); break;
    }
}

}  // namespace spamm
