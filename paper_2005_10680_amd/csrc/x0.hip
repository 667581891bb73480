// A1: the starting matrix of the purification.  Gerschgorin discs bound the
// spectrum of F by [lmin, lmax]; X_0 = (lmax I - F) / (lmax - lmin) maps it
// into [0, 1] with occupied states near 1.  X_0 has the block pattern of F
// plus every diagonal block.
#include <math.h>

#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

// per-row disc: centre f_rr, radius RN(sum_{c != r} |f_rc|), the exact sum
// rounded once.  One workgroup per block row I; thread t takes row r = t % b
// of the block row and the block columns J = t / b, t / b + P, ...
// (P = 256 / b), so each wave reads whole block columns (coalesced) and
// looks the block up once; the P double-double partial sums of a row are
// combined in a fixed order.  The high part is the rounded exact sum when
// the double-double value lies farther from a rounding boundary than its
// error bound (at most 2^18 positive terms: below 2^-87 of the sum); a row
// that misses the certificate gets lo[g] = NaN and its radius is summed
// exactly by launch_gersch_exact.
__global__ __launch_bounds__(256) void k_gersch_rows(MatView F, double* __restrict__ lo, double* __restrict__ hi) {
    __shared__ double shi[256], slo[256], scen[256];
    __shared__ int shas[256];
    const int64_t n = F.n;
    const int b = F.b, nb = F.nb;
    const int P = 256 / b;
    const int r = threadIdx.x % b, part = threadIdx.x / b;
    for (int I = blockIdx.x; I < nb; I += gridDim.x) {
        const int64_t g = (int64_t)I * b + r;
        dd rad = {0.0, 0.0};
        double cen = 0.0;
        bool has_cen = false, special = false, tiny = false;
        for (int J = part; J < nb; J += P) {
            const int s = F.map[(size_t)I * nb + J];
            if (s < 0) continue;
            const double* v = F.val + (size_t)s * b * b;
            // columns below n, in ascending order; sixteen loads in flight
            // before their additions
            const int64_t rem = n - (int64_t)J * b;
            const int cnt = rem < (int64_t)b ? (int)rem : b;
            for (int c0 = 0; c0 < cnt; c0 += 16) {
                double xs[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) xs[u] = c0 + u < cnt ? v[(size_t)(c0 + u) * b + r] : 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    if (c0 + u >= cnt) break;
                    const double x = xs[u];
                    if ((int64_t)J * b + c0 + u == g) {
                        cen = x;
                        has_cen = true;
                    } else {
                        const double ax = fabs(x);
                        if (!(ax < 0x1p1000)) special = true;           // huge, inf or NaN
                        else if (ax != 0.0 && ax < 0x1p-900) tiny = true;  // error terms may underflow
                        rad = dd_add(rad, dd{ax, 0.0});
                    }
                }
            }
        }
        shi[threadIdx.x] = rad.hi;
        slo[threadIdx.x] = rad.lo;
        scen[threadIdx.x] = cen;
        shas[threadIdx.x] = (has_cen ? 1 : 0) | (special ? 2 : 0) | (tiny ? 4 : 0);
        __syncthreads();
        if (part == 0 && g < n) {
            dd acc = {shi[r], slo[r]};
            double c0 = (shas[r] & 1) ? scen[r] : 0.0;
            int fl = shas[r];
            for (int q = 1; q < P; ++q) {
                acc = dd_add(acc, dd{shi[q * b + r], slo[q * b + r]});
                if (shas[q * b + r] & 1) c0 = scen[q * b + r];  // the part that met column g
                fl |= shas[q * b + r];
            }
            if (sq_certified(acc, (fl & 2) != 0, (fl & 4) != 0)) {
                lo[g] = c0 - acc.hi;
                hi[g] = c0 + acc.hi;
            } else {
                lo[g] = NAN;  // summed exactly by launch_gersch_exact
                hi[g] = c0;
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_gersch_final(const double* __restrict__ lo, const double* __restrict__ hi,
                                                      int64_t n, double* __restrict__ lam) {
    __shared__ double sl[1024], sh[1024];
    double a = INFINITY, z = -INFINITY;
    for (int64_t g = threadIdx.x; g < n; g += blockDim.x) {
        a = fmin(a, lo[g]);
        z = fmax(z, hi[g]);
    }
    sl[threadIdx.x] = a;
    sh[threadIdx.x] = z;
    __syncthreads();
    for (int st = 512; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sl[threadIdx.x] = fmin(sl[threadIdx.x], sl[threadIdx.x + st]);
            sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        lam[0] = sl[0];
        lam[1] = sh[0];
    }
}

void launch_gersch(const MatView& F, double* rowtmp, double* lam, hipStream_t s) {
    hipLaunchKernelGGL(k_gersch_rows, dim3(grid_for(F.nb, 1, 4096)), dim3(256), 0, s, F, rowtmp, rowtmp + F.n);
    launch_gersch_exact(F, rowtmp, rowtmp + F.n, s);
    hipLaunchKernelGGL(k_gersch_final, dim3(1), dim3(1024), 0, s, rowtmp, rowtmp + F.n, F.n, lam);
}

__global__ void k_x0_diagflags(MatView F, int32_t* __restrict__ flag) {
    for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < F.nb; d += gridDim.x * blockDim.x)
        flag[d] = F.map[(size_t)d * F.nb + d] < 0 ? 1 : 0;
}

__global__ void k_x0_meta(MatView F, MatView X, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                          const int64_t* __restrict__ nmiss) {
    int64_t nf = *F.nslot;
    if (nf > F.cap) nf = F.cap;
    const int64_t tot = nf + *nmiss;
    if (blockIdx.x == 0 && threadIdx.x == 0) *X.nslot = (int32_t)(tot <= X.cap ? tot : X.cap);
    const int nb = F.nb;
    const int64_t nn = (int64_t)nb * nb;
    const int64_t span = nn > nf ? nn : nf;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < span; t += (int64_t)gridDim.x * blockDim.x) {
        if (t < nf && t < X.cap) {
            X.brow[t] = F.brow[t];
            X.bcol[t] = F.bcol[t];
        }
        if (t < nn) X.map[t] = F.map[t];
    }
}

__global__ void k_x0_diagslots(MatView F, MatView X, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos) {
    int64_t nf = *F.nslot;
    if (nf > F.cap) nf = F.cap;
    for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < F.nb; d += gridDim.x * blockDim.x) {
        if (!flag[d]) continue;
        const int64_t s = nf + pos[d];
        if (s >= X.cap) continue;
        X.brow[s] = d;
        X.bcol[s] = d;
        X.map[(size_t)d * F.nb + d] = (int32_t)s;
    }
}

template <int B>
__global__ __launch_bounds__(256) void k_x0_vals(MatView F, MatView X, const double* __restrict__ lam) {
    int64_t nf = *F.nslot;
    if (nf > F.cap) nf = F.cap;
    int64_t nx = *X.nslot;
    if (nx > X.cap) nx = X.cap;
    const double lmin = lam[0], lmax = lam[1];
    const double W = lmax - lmin;
    const int64_t n = F.n;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t s = (int64_t)blockIdx.x * 4 + wv; s < nx; s += (int64_t)gridDim.x * 4) {
        const int r = X.brow[s];
        if (r < 0) continue;
        const int c = X.bcol[s];
        const double* src = s < nf ? F.val + (size_t)s * B * B : nullptr;
        double* dst = X.val + (size_t)s * B * B;
        for (int t = lane; t < B * B; t += 64) {
            const int col = t / B, row = t % B;
            const int64_t gi = (int64_t)r * B + row, gj = (int64_t)c * B + col;
            const double f = src ? src[t] : 0.0;
            double x;
            if (gi >= n || gj >= n) x = 0.0;
            else if (gi == gj) x = (lmax - f) / W;
            else x = (-f) / W;
            dst[t] = x;
        }
    }
}

void launch_x0(const MatView& F, const double* lam, const MatView& X, int32_t* diagflag, int32_t* diagpos,
               void* scan_temp, int64_t* tmp_count, hipStream_t s) {
    hipLaunchKernelGGL(k_x0_diagflags, dim3(grid_for(F.nb, 256, 64)), dim3(256), 0, s, F, diagflag);
    scan_i32(diagflag, diagpos, F.nb, nullptr, tmp_count, scan_temp, s);
    const int64_t nn = (int64_t)F.nb * F.nb;
    hipLaunchKernelGGL(k_x0_meta, dim3(grid_for(nn > F.cap ? nn : F.cap, 256, 4096)), dim3(256), 0, s, F, X, diagflag,
                       diagpos, tmp_count);
    hipLaunchKernelGGL(k_x0_diagslots, dim3(grid_for(F.nb, 256, 64)), dim3(256), 0, s, F, X, diagflag, diagpos);
    const int grid = grid_for(X.cap, 4, 4096);
    switch (F.b) {
        case 32: hipLaunchKernelGGL(k_x0_vals<32>, dim3(grid), dim3(256), 0, s, F, X, lam); break;
        case 64: hipLaunchKernelGGL(k_x0_vals<64>, dim3(grid), dim3(256), 0, s, F, X, lam); break;
        case 128: hipLaunchKernelGGL(k_x0_vals<128>, dim3(grid), dim3(256), 0, s, F, X, lam); break;
    }
}

}  // namespace spamm
