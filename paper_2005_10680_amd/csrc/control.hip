// The traces of the current iterate and the decisions the purification loop
// (Algorithms 1, 4, 5) takes from them.
//
// In the device-driven loop the decisions are taken by one thread on the
// device, so that a captured graph of the whole step can be replayed without
// reading anything back; in the host loop the same launch gathers what the
// host reads into host-mapped memory.  Both run in the traces launch itself,
// in its last workgroup.  Same rules, same arithmetic as the host (the
// shared sp2_* functions of common.hpp).
#include <algorithm>

#include "../../include/spamm.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

// One control step: record the results of the step that produced the current
// iterate, then (unless the loop stops) the next step's branch, delta_i and
// budgets.  tr: t1 hi, lo, t2 hi, lo of the current iterate.
SPAMM_DEV void sp2_control(Sp2Ctl* ctl_p, const double* tr, const int64_t* msc_p, const int64_t* ts_p,
                           const int32_t* ovf_mul, const int32_t* ovf_sweep, sp2_iter_log* logs,
                           int32_t max_records) {
    // everything read up front (independent loads in flight together), the
    // decisions in registers, the control block written back once
    Sp2Ctl c = *ctl_p;
    const int32_t ovf = *ovf_mul | *ovf_sweep;
    int64_t msc[4], ts[3];
    for (int q = 0; q < 4; ++q) msc[q] = msc_p[q];
    for (int q = 0; q < 3; ++q) ts[q] = ts_p[q];
    if (c.done) return;
    const int nlog = c.nlog;
    const int it = nlog + 1;
    if (ovf) {
        ctl_p->status = SPAMM_ECAPACITY;
        ctl_p->done = 1;
        return;
    }
    if (nlog > 0) {
        // results of the step that produced the current iterate
        sp2_iter_log& L = logs[nlog - 1];
        L.idx = c.idx;
        L.tau = c.tau;
        L.npairs = msc[0];
        L.nout = msc[1];
        L.nslot_hat = msc[2];
        L.removed_units = ts[0];
        L.removed_fro2 = (double)ts[1] * sp2_trunc_quantum(L.delta * c.trunc_scale);
        L.nslot_kept = msc[2] - ts[2];  // blocks of X~: those of X^ minus the removed ones
        L.npairs_low = c.tiered ? msc[3] : 0;
        L.sigma = c.sigma;
        L.sidx = c.sidx;
    }
    const double t1 = tr[0], t2 = tr[2];
    const double e = dd_diff(tr[0], tr[1], tr[2], tr[3]);
    c.e_hist[2] = c.e_hist[1];
    c.e_hist[1] = c.e_hist[0];
    c.e_hist[0] = e;
    if (c.n_e < 3) c.n_e += 1;
    if (nlog >= max_records) {  // cannot happen with n_max + 2 records; stop safely
        c.status = SPAMM_WNOCONV;
        c.done = 1;
        *ctl_p = c;
        return;
    }
    sp2_iter_log L = sp2_iter_log{};
    L.i = it;
    L.t1 = t1;
    L.t2 = t2;
    L.e = e;
    L.branch = -1;
    c.nlog = nlog + 1;
    const bool stop = sp2_should_stop(c.e_hist, c.n_e, c.e_tol);
    if (stop || it > c.n_max) {
        L.stop = stop ? 1 : 2;
        c.status = stop ? SPAMM_OK : SPAMM_WNOCONV;
        c.done = 1;
    } else {
        const int br = sp2_choose_branch(t1, t2, c.n_occ);
        if (c.have_gap) {
            c.xh = sp2_map_gap(c.xh, br);
            c.xl = sp2_map_gap(c.xl, br);
        }
        const double delta = sp2_step_delta(c.eps, c.n_max, c.delta_const, c.xh - c.xl);
        L.branch = br;
        L.delta = delta;
        c.branch = br;
        c.delta = delta;
        c.budget = c.variant == 0 ? delta / 2.0 : delta;
        c.budget_skip = c.tiered ? c.tier_split * c.budget : c.budget;
        c.tau = 0.0;
        c.idx = c.N;
        c.sigma = 0.0;
        c.sidx = c.N;
    }
    logs[nlog] = L;
    *ctl_p = c;
}

// ---------------------------------------------------------------------------
// Traces: t1 = sum of the diagonal entries (rows below n), t2 = sum over the
// live slots of (sq + sqlo) = ||X||_F^2, both in double-double.  A grid
// fixed by the matrix size and a fixed reduction order (slots strided over
// the grid, a wave tree, the four waves in order, then the partials of the
// workgroups: lane l adds partial l + 64 to partial l, then a wave tree), so
// the result depends only on the slot contents and order.
// ---------------------------------------------------------------------------
constexpr int kTrBlocks = 120;
static_assert(kTrBlocks <= 128, "two partials per lane in the last workgroup");

__global__ __launch_bounds__(256) void k_traces(const int32_t* __restrict__ nslot_p, int64_t cap, int b, int64_t n,
                                               const int32_t* __restrict__ brow, const int32_t* __restrict__ bcol,
                                               const double* __restrict__ val, const double* __restrict__ sq,
                                               const double* __restrict__ sqlo, double* part /* [kTrBlocks][4] */,
                                               double* __restrict__ out, const int32_t* __restrict__ done,
                                               TraceTail tail) {
    __shared__ double sh[4][4];
    __shared__ int s_last;
    if (done && *done) return;
    int64_t nslot = *nslot_p;
    if (nslot > cap) nslot = cap;
    dd d1 = {0, 0}, d2 = {0, 0};
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslot; s += (int64_t)gridDim.x * blockDim.x) {
        int r = brow[s];
        if (r < 0) continue;
        d2 = dd_add(d2, dd{sq[s], 0.0});
        d2 = dd_add(d2, dd{sqlo[s], 0.0});
        if (r == bcol[s]) {
            // diagonal entries t < cnt (rows below n), added in ascending t;
            // sixteen loads in flight before their additions
            const double* v = val + (size_t)s * b * b;
            const int64_t rem = n - (int64_t)r * b;
            const int cnt = rem < (int64_t)b ? (int)rem : b;
            for (int t0 = 0; t0 < cnt; t0 += 16) {
                double x[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) x[u] = t0 + u < cnt ? v[(size_t)(t0 + u) * b + t0 + u] : 0.0;
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (t0 + u < cnt) d1 = dd_add(d1, dd{x[u], 0.0});
            }
        }
    }
    d1 = dd_wave_sum(d1);
    d2 = dd_wave_sum(d2);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sh[w][0] = d1.hi; sh[w][1] = d1.lo; sh[w][2] = d2.hi; sh[w][3] = d2.lo;
    }
    __syncthreads();
    int32_t* ticket = reinterpret_cast<int32_t*>(part + kTrBlocks * 4);
    if (threadIdx.x == 0) {
        dd a = {0, 0}, c = {0, 0};
        for (int q = 0; q < 4; ++q) {
            a = dd_add(a, dd{sh[q][0], sh[q][1]});
            c = dd_add(c, dd{sh[q][2], sh[q][3]});
        }
        part[blockIdx.x * 4 + 0] = a.hi; part[blockIdx.x * 4 + 1] = a.lo;
        part[blockIdx.x * 4 + 2] = c.hi; part[blockIdx.x * 4 + 3] = c.lo;
        __threadfence();  // the partial is visible before the ticket is taken
        s_last = atomicAdd(ticket, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    // last workgroup: every partial is written
    __threadfence();
    if (threadIdx.x >= 64) return;
    const int G = (int)gridDim.x;
    dd a = {0, 0}, c = {0, 0};
    if (lane < G) {
        a = dd{part[lane * 4 + 0], part[lane * 4 + 1]};
        c = dd{part[lane * 4 + 2], part[lane * 4 + 3]};
    }
    if (lane + 64 < G) {
        a = dd_add(a, dd{part[(lane + 64) * 4 + 0], part[(lane + 64) * 4 + 1]});
        c = dd_add(c, dd{part[(lane + 64) * 4 + 2], part[(lane + 64) * 4 + 3]});
    }
    a = dd_wave_sum(a);
    c = dd_wave_sum(c);
    if (lane != 0) return;
    *ticket = 0;
    const double tr[4] = {a.hi, a.lo, c.hi, c.lo};
    out[0] = tr[0]; out[1] = tr[1]; out[2] = tr[2]; out[3] = tr[3];
    if (tail.ctl) sp2_control(tail.ctl, tr, tail.msc, tail.ts, tail.ovf_mul, tail.ovf_sweep, tail.logs,
                              tail.max_records);
    if (tail.hs) {
        // what the host loop reads after each step, into host-mapped memory
        Sp2HostStatus* o = tail.hs;
        for (int q = 0; q < 4; ++q) {
            o->tr[q] = tr[q];
            o->msc[q] = tail.msc[q];
        }
        o->ts[0] = tail.ts[0];
        o->ts[1] = tail.ts[1];
        o->ts[2] = tail.ts[2];
        o->ovf[0] = *tail.ovf_mul;
        o->ovf[1] = *tail.ovf_sweep;
        o->nslot = *nslot_p;
        o->ctl = *tail.ctl_read;
        __threadfence_system();
    }
}

size_t traces_temp_bytes() { return sizeof(double) * 4 * kTrBlocks + 64; }

__global__ void k_traces_init(double* part) {
    if (threadIdx.x == 0) *reinterpret_cast<int32_t*>(part + kTrBlocks * 4) = 0;
}

void launch_traces_init(double* temp, hipStream_t s) {
    hipLaunchKernelGGL(k_traces_init, dim3(1), dim3(64), 0, s, temp);
}

void launch_traces(const int32_t* nslot, int64_t cap, int b, int64_t n, const int32_t* brow, const int32_t* bcol,
                   const double* val, const double* sq, const double* sqlo, double* temp, double* out,
                   const int32_t* done, hipStream_t s, const TraceTail& tail) {
    // one workgroup per 256 block positions of the nb x nb grid, at most
    // kTrBlocks: a function of the matrix size only, so every run of one
    // system (host or device loop, alone or batched) adds in the same order
    const int64_t nb = (n + b - 1) / b;
    const int grid = (int)std::min<int64_t>(kTrBlocks, std::max<int64_t>(1, (nb * nb + 255) / 256));
    hipLaunchKernelGGL(k_traces, dim3(grid), dim3(256), 0, s, nslot, cap, b, n, brow, bcol, val, sq, sqlo, temp, out,
                       done, tail);
}

// The control block of the device-driven loop: the host's settings, and from
// the spectral bounds lam = (lambda_min, lambda_max) the gap edges mapped to
// [0, 1] and delta_0 (the host loop's arithmetic, in the same order).
__global__ void k_sp2_init(Sp2Ctl hc, const double* __restrict__ lam, Sp2Ctl* __restrict__ ctl) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double W = lam[1] - lam[0];
    hc.xh = hc.have_gap ? (lam[1] - hc.homo) / W : NAN;
    hc.xl = hc.have_gap ? (lam[1] - hc.lumo) / W : NAN;
    hc.delta = sp2_step_delta(hc.eps, hc.n_max, hc.delta_const, hc.xh - hc.xl);
    *ctl = hc;
}

void launch_sp2_init(const Sp2Ctl& hc, const double* lam, Sp2Ctl* ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_sp2_init, dim3(1), dim3(64), 0, s, hc, lam, ctl);
}

__global__ void k_ctl_upload(const Sp2Ctl* __restrict__ src, Sp2Ctl* __restrict__ ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctl = *src;
}

void launch_ctl_upload(const Sp2Ctl* src, Sp2Ctl* ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_upload, dim3(1), dim3(64), 0, s, src, ctl);
}

}  // namespace spamm
