// Internal launcher interface between the C ABI (api.hip) and the kernels.
#pragma once
#include "common.hpp"

struct sp2_iter_log;  // include/spamm.h

namespace spamm {

// A block-sparse matrix as the kernels see it (see spamm_bsm in spamm.h).
struct MatView {
    int64_t n;
    int32_t b, nb;
    int64_t cap;
    int32_t* nslot;
    int32_t* brow;
    int32_t* bcol;
    int32_t* map;
    double* val;
    double* norm;
    double* sq;
    double* sqlo;
};

// norms.hip
void launch_norms(int b, const int32_t* nslot, int64_t cap, const int32_t* brow, const double* val, double* sq,
                  double* sqlo, double* nrm, hipStream_t s, const int32_t* done = nullptr);
// dst <- src (slot count, block map, the live slots s < min(nslot, cap));
// dst holds at least cap slots
void launch_copy_live(const MatView& src, const MatView& dst, int64_t cap, hipStream_t s);
// norms of the *nlist slots in list (the blocks a producer could not certify)
void launch_norms_listed(int b, const int32_t* list, const int32_t* nlist, int64_t cap, const int32_t* brow,
                         const double* val, double* sq, double* sqlo, double* nrm, hipStream_t s,
                         const int32_t* done = nullptr);

// Rotation of row k of an FP32 copy (the ring kernel's layout): element m of
// row k (index k of the column-major block's columns) at position
// (m + f32_rot(k)) mod b.  A read of four consecutive rows (16 lanes each)
// then covers four different 16-float bank ranges; only k mod 4 matters.
template <int B>
SPAMM_DEV int f32_rot(int k) { return B == 64 ? 16 * (k & 3) : 16 * ((k >> 1) & 1); }

// Row bitmaps of A (bit k of row i: A_ik present) and column bitmaps of B
// (bit k of column j: B_kj present) turn the inner indices of output (i, j)
// into a word AND.
// Visit the kept inner indices of output (i, j) in ascending k.
template <typename F>
SPAMM_DEV void for_each_kept(int i, int j, int nb, int nw, const uint32_t* bitsA, const uint32_t* bitsB,
                             const int32_t* mapA, const double* normA, const int32_t* mapB, const double* normB,
                             int btrans, double tau, F&& f) {
    for (int w = 0; w < nw; ++w) {
        uint32_t m = bitsA[(size_t)i * nw + w] & bitsB[(size_t)j * nw + w];
        while (m) {
            int t = __ffs(m) - 1;
            m &= m - 1;
            int k = w * 32 + t;
            int sa = mapA[(size_t)i * nb + k];
            int sb = btrans ? mapB[(size_t)j * nb + k] : mapB[(size_t)k * nb + j];
            if (sa < 0 || sb < 0) continue;
            double p = normA[sa] * normB[sb];
            if (p >= tau) f(k, sa, sb, p);
        }
    }
}

// the FP32 tier takes a pair only when both block norms are at least this
// (entries and partial results below FP32's normal range then lose less than
// the rounding constant's underflow term covers)
constexpr double kFp32TierNormMin = 0x1p-40;

// pairs.hip
enum OccMode { kOccA = 0, kOccB = 1, kOccBt = 2 };
void launch_occupancy(const MatView& M, int mode, uint32_t* bits, int nw, uint8_t* tiles, int T, int l0,
                      const int32_t* done, hipStream_t s);
void launch_kept_count(int nb, int P, int nw, const uint32_t* bitsA, const uint32_t* bitsB, const int32_t* mapA,
                       const double* normA, const int32_t* mapB, const double* normB, int btrans, int sym,
                       const double* tau, const double* sigma, double norm_min, int32_t* cnt, int32_t* cnt_flag,
                       int32_t* cnt_low, const int32_t* done, hipStream_t s);
void launch_kept_fill(int nb, int P, int nw, const uint32_t* bitsA, const uint32_t* bitsB, const int32_t* mapA,
                      const double* normA, const int32_t* mapB, const double* normB, int btrans, const double* tau,
                      const double* sigma, double norm_min, const int32_t* cnt, const int32_t* off,
                      const int32_t* oidx, const int64_t* npairs, const int64_t* nout, int64_t cap_pairs,
                      int64_t cap_out, int32_t* oi, int32_t* oj, int32_t* optr, int2* pairs, int32_t* olow,
                      int32_t* ovf, const int32_t* done, hipStream_t s);
void launch_hat_flags(int nb, int P, const int32_t* cnt, int sym, const int32_t* mapX, const int32_t* branch,
                      int32_t* flag, const int32_t* done, hipStream_t s);
void launch_hat_assign(int nb, int P, const int32_t* cnt, int sym, const int32_t* flag, const int32_t* slot,
                       const int64_t* nslot_total, int64_t cap, int32_t* map, int32_t* brow, int32_t* bcol,
                       int32_t* nslot, uint8_t* fromc, int32_t* ovf, const int32_t* done, hipStream_t s);
// Block norm outputs of a kernel that writes blocks (all null: none); a
// slot whose rounding cannot be certified goes to recheck[(*nrecheck)++].
struct NormOut {
    double* sq = nullptr;
    double* sqlo = nullptr;
    double* nrm = nullptr;
    int32_t* recheck = nullptr;
    int32_t* nrecheck = nullptr;
};
void launch_rest(int b, const int32_t* nslot_hat, int64_t cap_hat, const int32_t* brow, const int32_t* bcol,
                 const uint8_t* fromc, int nb, const int32_t* mapX, const double* valX, double* valH,
                 const int32_t* branch, const int32_t* done, hipStream_t s, NormOut no = NormOut(),
                 float* out32 = nullptr);

// Small systems: the occupancy, sweep-list, kept-pair and output-pattern
// passes of one step, each in a single workgroup (same results, fewer
// dependent launches).  Used for nb <= kSmallNb while small_path_enabled().
constexpr int kSmallNb = 64;
constexpr int kSmallPP = kSmallNb * kSmallNb;  // output positions of the pair pass
constexpr int kSmallTiles = 16;                // level-l0 tiles per side of the sweep
bool small_path_enabled();
void set_small_path(bool on);
// bits (nb x nw words) and tiles (T x T) of X as k_occupancy with kOccA; with
// cube_keys also the sweep's cube list of X X^T and its length in *ncubes
void launch_occ_small(const MatView& X, uint32_t* bits, int nw, uint8_t* tiles, int T, int l0, uint32_t* cube_keys,
                      int64_t* ncubes, const int32_t* done, hipStream_t s);
// kept pairs, output list, output pattern of C and its slots, sc[0..3] as the
// device-wide passes, counters[0..15] = 0, and the ring kernel's 9 cuts
void launch_pairs_small(int nb, int P, int nw, const uint32_t* bitsA, const uint32_t* bitsB, const int32_t* mapA,
                        const double* normA, const int32_t* mapB, const double* normB, int btrans, int sym,
                        const double* tau, const double* sigma, double norm_min, int64_t cap_pairs, int64_t cap_out,
                        int32_t* oi, int32_t* oj, int32_t* optr, int2* pairs, int32_t* olow, int64_t* sc,
                        int64_t capC, int32_t* mapC, int32_t* browC, int32_t* bcolC, int32_t* nslotC,
                        uint8_t* fromc, const int32_t* mapX, const int32_t* branch, int32_t* counters,
                        int32_t* cuts, int32_t* ovf, const int32_t* done, hipStream_t s);

// cse.hip
size_t cse_cube_cap(int nb);
int cse_level0(int nb);
void launch_cube_flags(int T, const uint8_t* tilesA, const uint8_t* tilesB, int32_t* flag, const int32_t* done,
                       hipStream_t s);
void launch_cube_list(int T, const int32_t* flag, const int32_t* idx, uint32_t* keys, const int64_t* ncubes,
                      int64_t cap, int32_t* ovf, const int32_t* done, hipStream_t s);
void launch_cube_eval(int mode, int l0, int nb, const uint32_t* keys, const int64_t* ncubes, int64_t cap,
                      const int32_t* mapA, const double* normA, const int32_t* mapB, const double* normB, int btrans,
                      const double* tau, int N, const double* tau0, double c_low, double* vals, const int32_t* done,
                      hipStream_t s);
void launch_level_flags(const uint32_t* keys, const int64_t* n, int64_t cap, int32_t* flag, const int32_t* done,
                        hipStream_t s);
void launch_level_build(const uint32_t* keys, const int64_t* n, int64_t cap, const int32_t* flag,
                        const int32_t* pos, const int64_t* nparent, uint32_t* pkeys, int32_t* pstart,
                        const int32_t* done, hipStream_t s);
void launch_level_eval(const uint32_t* ckeys, const double* cvals, const int32_t* pstart, const int64_t* nparent,
                       int64_t cap, int N, double* pvals, const int32_t* done, hipStream_t s);
// the levels above one of at most kTopNodes nodes, and the selection, in one
// workgroup (nlev levels from the nodes keys / va; vb the other value buffer)
constexpr int kTopNodes = 4096;
void launch_levels_top(const uint32_t* keys, const int64_t* n, double* va, double* vb, int nlev, int N,
                       const double* tau, const double* budget_dev, double budget_host, double* bound_out,
                       int32_t* idx_out, double* tau_out, const int32_t* done, hipStream_t s);
void launch_select(const double* root, const int64_t* nroot, const double* tau, int N, const double* budget_dev,
                   double budget_host, double* bound_out, int32_t* idx_out, double* tau_out, const int32_t* done,
                   hipStream_t s);

// gemm.hip
struct GemmArgs {
    int b, nb;
    const int32_t* oi;
    const int32_t* oj;
    const int32_t* optr;
    // (slot in valA, slot in valB); with btrans, a pair whose first slot is
    // negative holds (~slot in valB, slot in valA) instead (FP64 pairs only)
    const int2* pairs;
    const int64_t* nout;
    const int64_t* npairs;
    const double* valA;
    const double* valB;
    int btrans;
    int sym;
    const int32_t* map_out;
    double* val_out;
    // combine with X (2X - C when *branch == 1); mapX/valX may be null
    const int32_t* mapX;
    const double* valX;
    const int32_t* branch;
    int32_t* counters;  // [16] work counters, reset by the launcher
    const int32_t* ovf; // nonzero: an earlier capacity overflow, skip
    const int32_t* done;
    // FP32 tier (null when off): FP32 copies of A and B, and per output the
    // number of low-tier pairs at the head of its pair list
    const float* valA32 = nullptr;
    const float* valB32 = nullptr;
    const int32_t* olow = nullptr;
    // split-BF16 tier (null when off): per slot the hi part (b*b bf16,
    // row-major) then the lo part, and the slot's power-of-two exponent
    const uint16_t* valA16 = nullptr;
    const uint16_t* valB16 = nullptr;
    const int32_t* expA = nullptr;
    const int32_t* expB = nullptr;
    // block norms of the written blocks (null when not wanted; ring kernels
    // only): sq, sqlo and norm of each slot written, as the norms kernel
    // defines them; a slot whose rounding cannot be certified from the
    // double-double sum is appended to recheck (count in *nrecheck) for the
    // norms kernel's listed mode
    double* sq_out = nullptr;
    double* sqlo_out = nullptr;
    double* nrm_out = nullptr;
    int32_t* recheck = nullptr;
    int32_t* nrecheck = nullptr;
    // FP32 copies of the written blocks in the ring kernel's layout (rows
    // rotated by f32_rot; null when not wanted; the FP32-tier kernels only),
    // for the next step's low tier
    float* out32 = nullptr;
    // the per-XCD output ranges of the ring kernel (9 cuts: the outputs whose
    // first pair lies below npairs * x / 8), when the pair pass computed them;
    // null: the kernel finds them itself
    const int32_t* cuts = nullptr;
};
// ev_start/ev_end (optional) are recorded right around the product kernel.
// counters_clear: the work counters g.counters[0..15] are already zero (the
// small-system pair pass clears them), so the reset launch is skipped
void launch_gemm_f64(const GemmArgs& g, int num_cu, hipStream_t s, hipEvent_t ev_start = nullptr,
                     hipEvent_t ev_end = nullptr, bool counters_clear = false);
// workgroups per CU of the ring kernels' persistent grid, by leaf size
int get_ring_per_cu(int b);
void set_ring_per_cu(int b, int per_cu);
// several products in one launch: descs_dev[nsys] on the device, out_off and
// pair_off [nsys + 1] scratch, counters [16]
void launch_gemm_batch(int b, int low, const GemmArgs* descs_dev, int nsys, int64_t* out_off, int64_t* pair_off,
                       int32_t* counters, int num_cu, hipStream_t s);
// split-BF16 copies of the live blocks: x = 2^e (hi + lo + err), max |x| 2^-e
// in [1, 2), hi = RN_bf16, lo = RN_bf16(x 2^-e - hi); row-major per slot;
// one workgroup per block, at most max_wg workgroups
void launch_to_bf16x2(int b, const int32_t* nslot, int64_t cap, const int32_t* brow, const double* val, uint16_t* out,
                      int32_t* expo, const int32_t* done, hipStream_t s, int max_wg = 8192);
// FP32 copies; swz = 1: rows rotated for the ring kernel (leaf 32 and 64), 0: the block's own layout
void launch_to_f32(int b, const int32_t* nslot, int64_t cap, const int32_t* brow, const double* val, float* out,
                   int swz, const int32_t* done, hipStream_t s);

// adjoint.hip
void launch_sym_half(const MatView& D, const double* dval, double* gval, hipStream_t s);
void launch_adj_outputs(const MatView& X, int32_t* flag, int32_t* pos, int32_t* oi, int32_t* oj, int64_t* nout,
                        void* scan_tmp, hipStream_t s);
void launch_adj_pairs(int nb, int nw, int64_t cap_out, const int64_t* nout, const int32_t* oi, const int32_t* oj,
                      const uint32_t* bitsX, const uint32_t* bitsG, const int32_t* mapX, const double* normX,
                      const int32_t* mapG, double tau, int32_t* cnt, int32_t* optr, int64_t* npairs,
                      int64_t cap_pairs, int2* pairs, int32_t* ovf, void* scan_tmp, hipStream_t s);
void launch_adj_fbar(const MatView& F, const int32_t* map0, const double* g0, const double* lam, double* fbar,
                     hipStream_t s);

// bounds.hip: leaf-level bounds B_flat (flat = 1) / B_sum (flat = 0) for the N
// candidates into out [N] (mode 1: tier mode, tau0 the fixed skip threshold,
// c_low the low tier's per-pair factor), exactly rounded sums over the
// outputs; scratch holds bound_leaf_scratch_bytes(nb, N) bytes
constexpr int kBoundMaxNb = 2048;
int64_t bound_part_waves(int nb);
size_t bound_leaf_scratch_bytes(int nb, int N);
void launch_bound_leaf(int nb, int nw, const uint32_t* bitsA, const uint32_t* bitsB, const int32_t* mapA,
                       const double* normA, const int32_t* mapB, const double* normB, int btrans, const double* tau,
                       int N, int flat, int mode, const double* tau0, double c_low, void* scratch, double* out,
                       const int32_t* done, hipStream_t s);

// control.hip
// What the host loop reads back after each step, gathered by one thread into
// host-mapped (pinned, coherent) memory in place of separate small copies.
struct Sp2HostStatus {
    double tr[4];      // traces of the current iterate (double-double t1, t2)
    int64_t msc[4];    // kept pairs, outputs, slots of X^, low-tier pairs
    int64_t ts[3];     // truncation: removed units, removed key sum, removed blocks
    int32_t ovf[2];    // capacity flags of the product and of the sweep
    int32_t nslot;     // slots of the current iterate
    int32_t pad;
    Sp2Ctl ctl;
    Sp2Ctl ctl_in;     // the host's decisions for the next step (uploaded by a kernel)
};
// *ctl = *src, src in host-mapped memory
void launch_ctl_upload(const Sp2Ctl* src, Sp2Ctl* ctl, hipStream_t s);
// *ctl = hc with xh, xl (gap edges mapped by the bounds lam[2] on the device)
// and delta_0 filled in
void launch_sp2_init(const Sp2Ctl& hc, const double* lam, Sp2Ctl* ctl, hipStream_t s);
// What runs after the traces of the current iterate, in the traces launch
// itself (by its last workgroup): the device control step (ctl set: graph
// loop) or the host-status gather (hs set: host loop), reading the previous
// step's results msc / ts / overflow flags.
struct TraceTail {
    Sp2Ctl* ctl = nullptr;             // control step on this block
    Sp2HostStatus* hs = nullptr;       // host-status gather into this record
    const Sp2Ctl* ctl_read = nullptr;  // hs: the control block it copies
    const int64_t* msc = nullptr;
    const int64_t* ts = nullptr;
    const int32_t* ovf_mul = nullptr;
    const int32_t* ovf_sweep = nullptr;
    ::sp2_iter_log* logs = nullptr;
    int max_records = 0;
};
// Traces t1 = tr(X) (rows below n) and t2 = ||X||_F^2 in double-double into
// out[4] (t1 hi, lo, t2 hi, lo), then the tail.  temp: traces_temp_bytes(),
// its completion counter cleared once by launch_traces_init before the first
// launch (every launch leaves it cleared).
size_t traces_temp_bytes();
void launch_traces_init(double* temp, hipStream_t s);
void launch_traces(const int32_t* nslot, int64_t cap, int b, int64_t n, const int32_t* brow, const int32_t* bcol,
                   const double* val, const double* sq, const double* sqlo, double* temp, double* out,
                   const int32_t* done, hipStream_t s, const TraceTail& tail = TraceTail());

// reblock.hip: Y (leaf Y.b, same n) from X; flag/pos [P^2] with P the power
// of two >= Y.nb, total: device int64, ovf: set when Y.cap is too small
void launch_reblock(const MatView& X, const MatView& Y, int32_t* flag, int32_t* pos, int64_t* total, void* scan_tmp,
                    int32_t* ovf, hipStream_t s);

// trunc.hip
size_t trunc_temp_bytes(int64_t cap);
// iterates of at most this many slots are truncated by one workgroup (the
// candidate keys in LDS) while small_path_enabled()
constexpr int64_t kTruncSmallCap = 4096;
struct TruncNoallocScratch {
    void* temp;      // truncation temporaries for up to trunc_noalloc_max_cap() slots
    int64_t* stats;  // [4]
    int32_t* ovf;    // [4]
};
int64_t trunc_noalloc_max_cap();
hipError_t trunc_noalloc_scratch(TruncNoallocScratch* out);
void launch_truncate(const MatView& X, const double* delta_dev, double delta_host, double delta_scale,
                     void* temp, int64_t cap, int64_t* stats /* [4] */, int32_t* ovf, const int32_t* done,
                     hipStream_t s);

// x0.hip
void launch_gersch(const MatView& F, double* rowtmp /* [nb*b*2] */, double* lam /* [2] */, hipStream_t s);
// rows whose radius the double-double sums left uncertified (lo[g] NaN, hi[g] the centre): exact radius
void launch_gersch_exact(const MatView& F, double* lo, double* hi, hipStream_t s);
void launch_x0(const MatView& F, const double* lam, const MatView& X, int32_t* diagflag, int32_t* diagpos,
               void* scan_temp, int64_t* tmp_count, hipStream_t s);

}  // namespace spamm
