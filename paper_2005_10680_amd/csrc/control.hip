// Device-side control of the purification loop (Algorithms 1, 4, 5): the
// decisions the host loop takes between two steps, taken by one thread on
// the device so that a captured graph of the whole step can be replayed
// without reading anything back.  Same rules, same arithmetic (the shared
// sp2_* functions of common.hpp).
#include "../../include/spamm.h"
#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

__global__ void k_sp2_control(Sp2Ctl* __restrict__ ctl, const double* __restrict__ tr,
                              const int64_t* __restrict__ msc, const int64_t* __restrict__ ts,
                              const int32_t* __restrict__ ovf_mul, const int32_t* __restrict__ ovf_sweep,
                              const int32_t* __restrict__ nslot_cur, sp2_iter_log* __restrict__ logs,
                              int32_t max_records) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (ctl->done) return;
    const int nlog = ctl->nlog;
    const int it = nlog + 1;
    if (*ovf_mul || *ovf_sweep) {
        ctl->status = SPAMM_ECAPACITY;
        ctl->done = 1;
        return;
    }
    if (nlog > 0) {
        // results of the step that produced the current iterate
        sp2_iter_log& L = logs[nlog - 1];
        L.idx = ctl->idx;
        L.tau = ctl->tau;
        L.npairs = msc[0];
        L.nout = msc[1];
        L.nslot_hat = msc[2];
        L.removed_units = ts[0];
        L.removed_fro2 = (double)ts[1] * sp2_trunc_quantum(L.delta * ctl->trunc_scale);
        L.nslot_kept = msc[2] - ts[2];  // blocks of X~: those of X^ minus the removed ones
        L.npairs_low = ctl->tiered ? msc[3] : 0;
        L.sigma = ctl->sigma;
        L.sidx = ctl->sidx;
    }
    const double t1 = tr[0], t2 = tr[2];
    const double e = dd_diff(tr[0], tr[1], tr[2], tr[3]);
    ctl->e_hist[2] = ctl->e_hist[1];
    ctl->e_hist[1] = ctl->e_hist[0];
    ctl->e_hist[0] = e;
    if (ctl->n_e < 3) ctl->n_e += 1;
    if (nlog >= max_records) {  // cannot happen with n_max + 2 records; stop safely
        ctl->status = SPAMM_WNOCONV;
        ctl->done = 1;
        return;
    }
    sp2_iter_log& L = logs[nlog];
    L = sp2_iter_log{};
    L.i = it;
    L.t1 = t1;
    L.t2 = t2;
    L.e = e;
    L.branch = -1;
    ctl->nlog = nlog + 1;
    const bool stop = sp2_should_stop(ctl->e_hist, ctl->n_e, ctl->e_tol);
    if (stop || it > ctl->n_max) {
        L.stop = stop ? 1 : 2;
        ctl->status = stop ? SPAMM_OK : SPAMM_WNOCONV;
        ctl->done = 1;
        return;
    }
    const int br = sp2_choose_branch(t1, t2, ctl->n_occ);
    if (ctl->have_gap) {
        ctl->xh = sp2_map_gap(ctl->xh, br);
        ctl->xl = sp2_map_gap(ctl->xl, br);
    }
    const double delta = sp2_step_delta(ctl->eps, ctl->n_max, ctl->delta_const, ctl->xh - ctl->xl);
    L.branch = br;
    L.delta = delta;
    ctl->branch = br;
    ctl->delta = delta;
    ctl->budget = ctl->variant == 0 ? delta / 2.0 : delta;
    ctl->budget_skip = ctl->tiered ? ctl->tier_split * ctl->budget : ctl->budget;
    ctl->tau = 0.0;
    ctl->idx = ctl->N;
    ctl->sigma = 0.0;
    ctl->sidx = ctl->N;
}

__global__ void k_host_status(const double* __restrict__ tr, const int64_t* __restrict__ msc,
                              const int64_t* __restrict__ ts, const int32_t* __restrict__ ovf_mul,
                              const int32_t* __restrict__ ovf_sweep, const Sp2Ctl* __restrict__ ctl,
                              const int32_t* __restrict__ nslot, Sp2HostStatus* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int q = 0; q < 4; ++q) {
        out->tr[q] = tr[q];
        out->msc[q] = msc[q];
    }
    out->ts[0] = ts[0];
    out->ts[1] = ts[1];
    out->ts[2] = ts[2];
    out->ovf[0] = *ovf_mul;
    out->ovf[1] = *ovf_sweep;
    out->nslot = *nslot;
    out->ctl = *ctl;
    __threadfence_system();
}

void launch_host_status(const double* tr, const int64_t* msc, const int64_t* ts, const int32_t* ovf_mul,
                        const int32_t* ovf_sweep, const Sp2Ctl* ctl, const int32_t* nslot, Sp2HostStatus* out,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_host_status, dim3(1), dim3(64), 0, s, tr, msc, ts, ovf_mul, ovf_sweep, ctl, nslot, out);
}

__global__ void k_ctl_upload(const Sp2Ctl* __restrict__ src, Sp2Ctl* __restrict__ ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctl = *src;
}

void launch_ctl_upload(const Sp2Ctl* src, Sp2Ctl* ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_upload, dim3(1), dim3(64), 0, s, src, ctl);
}

void launch_sp2_control(Sp2Ctl* ctl, const double* tr, const int64_t* msc, const int64_t* ts, const int32_t* ovf_mul,
                        const int32_t* ovf_sweep, const int32_t* nslot_cur, sp2_iter_log* logs, int max_records,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_sp2_control, dim3(1), dim3(64), 0, s, ctl, tr, msc, ts, ovf_mul, ovf_sweep, nslot_cur, logs,
                       max_records);
}

}  // namespace spamm
