// K3: leaf products of the kept pairs (the "lowest level" of Algorithm 2)
// on the CDNA matrix cores, FP64 with an optional FP32 precision tier.
//
// One workgroup (4 waves) owns one output block C_ij = sum_k A_ik B_kj and
// walks its kept pairs in list order (ascending k inside each tier).  The
// inner dimension of all pairs is streamed in chunks of KC: the A chunk (KC
// columns of the column-major A_ik) and the B chunk (KC rows of B_kj) are
// staged through a double-buffered LDS tile while the next chunk is in
// flight.  Each wave accumulates a (B/2) x (B/2) quadrant.
//
// Precision tiers: an output's list holds its low-tier pairs first.  Those
// use FP32 copies of the blocks and V_MFMA_F32_16X16X4_F32; the FP32 result
// of each pair is added into an FP64 accumulator before the next pair
// starts, so every pair's rounding error stays within c_32 * ||A_ik|| ||B_kj||
// (the factor the sweep folds into its bound).  The remaining pairs use
// V_MFMA_F64_16X16X4_F64.
//
// Epilogue: the accumulators go through an LDS tile (the two MFMA result
// layouts differ: FP64 register r of lane l holds row (l>>4) + 4r, FP32
// holds row 4(l>>4) + r, column l&15 in both), the SP2 combine
// (X^ = C or 2X - C) is applied once, and the block and, in symmetric
// mode, its mirror C_ji = C_ij^T are written with coalesced stores.
//
// The kernel is persistent: the grid is a multiple of the 8 XCDs, the output
// list (Morton order) is cut into 8 contiguous ranges of equal kept-pair
// count, and the workgroups of XCD x take outputs of range x from an atomic
// counter, so neighbouring outputs -- which share A rows and B columns --
// run under the same L2.  In the ring kernels (k_gemm_ring, k_gemm_ring_batch)
// a workgroup whose range is drained goes on with the other ranges' counters,
// so the XCDs finish together; the register-staged k_gemm (B not given
// transposed) stops at the end of its own range.  Every output is computed by
// exactly one workgroup in a fixed order: results are bitwise reproducible.
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace spamm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <int B>
struct GemmCfg {
    static constexpr int TM = B / 32;  // 16x16 tiles per wave along rows (2 waves)
    static constexpr int TN = B / 32;  // along columns (2 waves)
    static constexpr int KC = 16;      // inner indices per LDS stage
    static constexpr int CH = B / KC;  // stages per kept pair
    static constexpr int LD = B + 4;   // LDS row stride of the staging tiles (elements)
    static constexpr int V2PT = KC * B / 2 / 256;  // 2-element loads per thread per operand
    static constexpr int PC = B < 64 ? B : 64;     // epilogue columns per pass
    static constexpr int NPASS = B / PC;
    static constexpr int LDT = B + 1;              // epilogue tile stride (doubles)
    static constexpr int STAGE_BYTES = 2 * 2 * KC * LD * 8;
    static constexpr int TILE_BYTES = PC * LDT * 8;
    static constexpr int LDS_BYTES = STAGE_BYTES > TILE_BYTES ? STAGE_BYTES : TILE_BYTES;
};

template <int N>
struct DVec {
    typedef double type __attribute__((ext_vector_type(N)));
};
template <int N>
struct FVec {
    typedef float type __attribute__((ext_vector_type(N)));
};
template <int B>
using StageD = typename DVec<2 * GemmCfg<B>::V2PT>::type;
template <int B>
using StageF = typename FVec<2 * GemmCfg<B>::V2PT>::type;

// Global -> register stage of one chunk (E = double or float).  The A chunk
// is KC contiguous columns of A_ik; the B chunk is KC contiguous columns of
// Bt_jk (BT) or KC rows of the column-major B_kj.
template <int B, bool BT, typename E, typename V>
SPAMM_DEV void load_stage(V& sa, V& sb, const E* __restrict__ valA, const E* __restrict__ valB, int2 pr, int chunk) {
    using C = GemmCfg<B>;
    using E2 = typename std::conditional<sizeof(E) == 8, double2, float2>::type;
    const int t = threadIdx.x;
    const E* a0 = valA + (size_t)pr.x * B * B + (size_t)chunk * C::KC * B;
#pragma unroll
    for (int v = 0; v < C::V2PT; ++v) {
        const E2 x = reinterpret_cast<const E2*>(a0)[t + 256 * v];
        sa[2 * v] = x.x;
        sa[2 * v + 1] = x.y;
    }
    if constexpr (BT) {
        const E* b0 = valB + (size_t)pr.y * B * B + (size_t)chunk * C::KC * B;
#pragma unroll
        for (int v = 0; v < C::V2PT; ++v) {
            const E2 x = reinterpret_cast<const E2*>(b0)[t + 256 * v];
            sb[2 * v] = x.x;
            sb[2 * v + 1] = x.y;
        }
    } else {
        const E* b0 = valB + (size_t)pr.y * B * B + (size_t)chunk * C::KC;
#pragma unroll
        for (int v = 0; v < C::V2PT; ++v) {
            const int idx = t + 256 * v;
            const int col = idx / (C::KC / 2), kp = idx % (C::KC / 2);
            const E2 x = *reinterpret_cast<const E2*>(b0 + (size_t)col * B + 2 * kp);
            sb[2 * v] = x.x;
            sb[2 * v + 1] = x.y;
        }
    }
}

// Register -> LDS: both tiles are stored [k][row or column].
template <int B, bool BT, typename E, typename V>
SPAMM_DEV void store_stage(const V& sa, const V& sb, E* As, E* Bs) {
    using C = GemmCfg<B>;
    using E2 = typename std::conditional<sizeof(E) == 8, double2, float2>::type;
    const int t = threadIdx.x;
#pragma unroll
    for (int v = 0; v < C::V2PT; ++v) {
        const int e = 2 * (t + 256 * v);
        const int k = e / B, r = e % B;
        *reinterpret_cast<E2*>(As + k * C::LD + r) = E2{sa[2 * v], sa[2 * v + 1]};
    }
    if constexpr (BT) {
#pragma unroll
        for (int v = 0; v < C::V2PT; ++v) {
            const int e = 2 * (t + 256 * v);
            const int k = e / B, c = e % B;
            *reinterpret_cast<E2*>(Bs + k * C::LD + c) = E2{sb[2 * v], sb[2 * v + 1]};
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

template <int B, bool BT, int LOWT>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    using C = GemmCfg<B>;
    __shared__ __attribute__((aligned(16))) char lds_raw[C::LDS_BYTES];
    __shared__ int s_o, s_lo, s_hi;
    if (g.done && *g.done) return;
    if (g.ovf && *g.ovf) return;
    double* ldsd = reinterpret_cast<double*>(lds_raw);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int64_t nout = *g.nout;
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
    const bool beta = g.mapX && g.branch && (*g.branch == 1);
    // staging buffers: [buf][A or B] regions of KC*LD doubles each
    char* const stg = lds_raw;
    constexpr size_t SB = (size_t)C::KC * C::LD * 8;

    while (true) {
        if (tid == 0) s_o = lo + atomicAdd(&g.counters[xcd], 1);
        __syncthreads();
        const int o = s_o;
        __syncthreads();
        if (o >= hi) break;
        const int i = g.oi[o], j = g.oj[o];
        const int p0 = g.optr[o], p1 = g.optr[o + 1];
        const int nlow = LOWT ? g.olow[o] : 0;
        const int nch = (p1 - p0) * C::CH;
        const int nch_low = nlow * C::CH;

        d4 acc[C::TM][C::TN];
        d4 dlow[C::TM][C::TN];  // FP64 sum of the low-tier pairs (FP32 result layout)
        f4 acc32[C::TM][C::TN];
#pragma unroll
        for (int a = 0; a < C::TM; ++a)
#pragma unroll
            for (int b = 0; b < C::TN; ++b) {
                acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
                if constexpr (LOWT != 0) {
                    dlow[a][b] = d4{0.0, 0.0, 0.0, 0.0};
                    acc32[a][b] = f4{0.f, 0.f, 0.f, 0.f};
                }
            }

        StageD<B> sa, sb;
        StageF<B> fa, fb;
        if (nch > 0) {
            const int2 pr = g.pairs[p0];
            if (LOWT && 0 < nch_low) {
                load_stage<B, BT, float>(fa, fb, g.valA32, g.valB32, pr, 0);
                store_stage<B, BT, float>(fa, fb, (float*)(stg), (float*)(stg + SB));
            } else {
                load_stage<B, BT, double>(sa, sb, g.valA, g.valB, pr, 0);
                store_stage<B, BT, double>(sa, sb, (double*)(stg), (double*)(stg + SB));
            }
        }
        __syncthreads();
        for (int gi = 0; gi < nch; ++gi) {
            const int buf = gi & 1;
            const bool low_now = LOWT && gi < nch_low;
            const bool low_next = LOWT && (gi + 1) < nch_low;
            if (gi + 1 < nch) {
                const int2 pr = g.pairs[p0 + (gi + 1) / C::CH];
                if (low_next) load_stage<B, BT, float>(fa, fb, g.valA32, g.valB32, pr, (gi + 1) % C::CH);
                else load_stage<B, BT, double>(sa, sb, g.valA, g.valB, pr, (gi + 1) % C::CH);
            }
            if constexpr (LOWT != 0) {
                if (low_now) {
                    const float* As = (const float*)(stg + (size_t)(2 * buf) * SB);
                    const float* Bs = (const float*)(stg + (size_t)(2 * buf + 1) * SB);
#pragma unroll
                    for (int ks = 0; ks < C::KC / 4; ++ks) {
                        const int kr = ks * 4 + (lane >> 4);
                        float av[C::TM], bv[C::TN];
#pragma unroll
                        for (int a = 0; a < C::TM; ++a) av[a] = As[kr * C::LD + wm * C::TM * 16 + a * 16 + (lane & 15)];
#pragma unroll
                        for (int b = 0; b < C::TN; ++b) bv[b] = Bs[kr * C::LD + wn * C::TN * 16 + b * 16 + (lane & 15)];
#pragma unroll
                        for (int a = 0; a < C::TM; ++a)
#pragma unroll
                            for (int b = 0; b < C::TN; ++b)
                                acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc32[a][b], 0, 0, 0);
                    }
                    if ((gi % C::CH) == C::CH - 1) {
                        // end of one low-tier pair: fold its FP32 product into FP64
#pragma unroll
                        for (int a = 0; a < C::TM; ++a)
#pragma unroll
                            for (int b = 0; b < C::TN; ++b) {
#pragma unroll
                                for (int r = 0; r < 4; ++r) dlow[a][b][r] = dlow[a][b][r] + (double)acc32[a][b][r];
                                acc32[a][b] = f4{0.f, 0.f, 0.f, 0.f};
                            }
                    }
                }
            }
            if (!low_now) {
                const double* As = (const double*)(stg + (size_t)(2 * buf) * SB);
                const double* Bs = (const double*)(stg + (size_t)(2 * buf + 1) * SB);
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
            }
            if (gi + 1 < nch) {
                char* nA = stg + (size_t)(2 * (buf ^ 1)) * SB;
                char* nB = stg + (size_t)(2 * (buf ^ 1) + 1) * SB;
                if (low_next) store_stage<B, BT, float>(fa, fb, (float*)nA, (float*)nB);
                else store_stage<B, BT, double>(sa, sb, (double*)nA, (double*)nB);
            }
            __syncthreads();
        }

        // ---------------- epilogue through LDS ----------------
        const int sh = g.map_out[(size_t)i * g.nb + j];
        const int sht = (g.sym && i != j) ? g.map_out[(size_t)j * g.nb + i] : -1;
        const int sx = beta ? g.mapX[(size_t)i * g.nb + j] : -1;
        double* dst = sh >= 0 ? g.val_out + (size_t)sh * B * B : nullptr;
        double* dstt = sht >= 0 ? g.val_out + (size_t)sht * B * B : nullptr;
        const double* xs = sx >= 0 ? g.valX + (size_t)sx * B * B : nullptr;
#pragma unroll
        for (int pass = 0; pass < C::NPASS; ++pass) {
            const int c0 = pass * C::PC;
            // FP64 accumulators: register r of lane l = row (l >> 4) + 4 r
#pragma unroll
            for (int a = 0; a < C::TM; ++a)
#pragma unroll
                for (int b = 0; b < C::TN; ++b) {
                    const int col = wn * C::TN * 16 + b * 16 + (lane & 15);
                    if (col < c0 || col >= c0 + C::PC) continue;
                    const int rowb = wm * C::TM * 16 + a * 16 + (lane >> 4);
#pragma unroll
                    for (int r = 0; r < 4; ++r) ldsd[(col - c0) * C::LDT + rowb + 4 * r] = acc[a][b][r];
                }
            if constexpr (LOWT != 0) {
                if (nlow > 0) {
                    __syncthreads();
                    // low-tier sums: register r of lane l = row 4 (l >> 4) + r
#pragma unroll
                    for (int a = 0; a < C::TM; ++a)
#pragma unroll
                        for (int b = 0; b < C::TN; ++b) {
                            const int col = wn * C::TN * 16 + b * 16 + (lane & 15);
                            if (col < c0 || col >= c0 + C::PC) continue;
                            const int rowb = wm * C::TM * 16 + a * 16 + 4 * (lane >> 4);
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                double* p = &ldsd[(col - c0) * C::LDT + rowb + r];
                                *p = *p + dlow[a][b][r];
                            }
                        }
                }
            }
            __syncthreads();
            // combine and write the block (coalesced along columns)
            for (int e = tid; e < C::PC * B; e += 256) {
                const int cl = e / B, row = e % B;
                double v = ldsd[cl * C::LDT + row];
                if (beta) {
                    const double x = xs ? xs[(size_t)(c0 + cl) * B + row] : 0.0;
                    v = 2.0 * x - v;
                    ldsd[cl * C::LDT + row] = v;
                }
                if (dst) dst[(size_t)(c0 + cl) * B + row] = v;
            }
            if (dstt) {
                __syncthreads();
                // mirror block: element (r', c') = C(c', r'); r' runs over this pass
                for (int e = tid; e < C::PC * B; e += 256) {
                    const int cp = e / C::PC, rp = e % C::PC;
                    dstt[(size_t)cp * B + c0 + rp] = ldsd[rp * C::LDT + cp];
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Transposed-B layout (the symmetric square and the adjoint products): both
// operand chunks are contiguous, so they are copied global -> LDS directly
// (global_load_lds_dwordx4, 16 B per lane, lane-contiguous) into a ring of NS
// stages, NS - 1 stages in flight while one is multiplied; no staging
// registers.  An FP32-tier stage covers 32 inner indices, an FP64 stage 16,
// so every stage moves the same bytes and every wave issues the same number
// of copies per stage: the wait before a stage is a fixed vmcnt.
// ---------------------------------------------------------------------------
template <int B>
struct RingCfg {
    static constexpr int KC64 = 16, KC32 = 32;
    static constexpr int CH64 = B / KC64, CH32 = B / KC32;
    static constexpr int OPB = KC64 * B * 8;           // bytes per operand chunk
    static constexpr int STAGE = 2 * OPB;              // A chunk then B chunk
    static constexpr int NS = B == 32 ? 4 : (B == 64 ? 3 : 2);
    static constexpr int NI = OPB / 1024 / 4;          // copies per wave per operand (1 KB per copy)
    static constexpr int PC = B == 128 ? 32 : B;       // epilogue columns per pass
    static constexpr int NPASS = B / PC;
    static constexpr int LDT = B + 1;
    static constexpr int TM = B / 32, TN = B / 32;
    // waves per SIMD the register allocation aims for (LDS allows 3
    // workgroups per CU at leaf 64)
    template <int LOWT>
    static constexpr int waves() { return B == 32 ? 4 : (B == 64 ? 3 : 1); }
};

template <int V>
SPAMM_DEV void wait_vmcnt() {
    static_assert(V >= 0 && V < 64, "vmcnt range");
    // gfx9 s_waitcnt: vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt_hi[15:14]
    __builtin_amdgcn_s_waitcnt((V & 0xF) | (0x7 << 4) | (0xF << 8) | (((V >> 4) & 0x3) << 14));
}

// copy one operand chunk (OPB contiguous bytes) into LDS; wave w takes the
// 1 KB pieces w, w+4, ...
template <int B>
SPAMM_DEV void dma_chunk(const char* __restrict__ src, char* lds_dst) {
    using R = RingCfg<B>;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < R::NI; ++q) {
        const int piece = w + 4 * q;
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void*)(src + (size_t)piece * 1024 + lane * 16),
            (__attribute__((address_space(3))) void*)(lds_dst + piece * 1024), 16, 0, 0);
    }
}

// Row rotation of the FP64 LDS tiles at leaf 32: row k (32 doubles, one
// 256 B bank period) holds its source row rotated by 16 doubles when k is
// odd, so the two k rows that 32 lanes of an operand read touch fall in
// different bank halves.  Leaf 64 reads two 16-column tiles per row with one
// ds_read2_b64 and keeps the plain layout.
SPAMM_DEV int f64_rot32(int k) { return 16 * (k & 1); }

// dma_chunk with the leaf-32 FP64 row rotation: each lane fetches the source
// 16 bytes that belong at its LDS position
template <int B>
SPAMM_DEV void dma_chunk_rot(const char* __restrict__ src, char* lds_dst) {
    static_assert(B == 32, "the rotation is for leaf 32");
    using R = RingCfg<B>;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < R::NI; ++q) {
        const int piece = w + 4 * q;
        const int pos = piece * 1024 + lane * 16;            // LDS byte offset in the chunk
        const int r = pos / (B * 8), p = (pos % (B * 8)) / 8;  // row, first of the lane's two doubles
        const int sp = (p - f64_rot32(r)) & (B - 1);
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void*)(src + (size_t)r * B * 8 + (size_t)sp * 8),
            (__attribute__((address_space(3))) void*)(lds_dst + piece * 1024), 16, 0, 0);
    }
}

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Row rotation of the split-BF16 LDS tiles: group g of row r sits at
// position (g + r/4) mod 4 of its 64 B row, so the 16 rows one MFMA operand
// read touches fall in 16 different bank quads.
SPAMM_DEV int bf16_rot(int r) { return (r >> 2) & 3; }

// Copy inner indices 32c .. 32c+31 of one split-BF16 block (hi part, then lo
// part, each b rows of b bf16, row-major) into LDS: per part b rows of four
// 16 B groups (8 inner indices each), rotated by bf16_rot.  Every 1 KB piece
// is 64 lane-contiguous 16 B copies, as the direct-to-LDS copy requires;
// each lane picks the global source of its LDS position.
template <int B>
SPAMM_DEV void dma_bf16_chunk(const char* __restrict__ blk, int chunk, char* lds_dst) {
    using R = RingCfg<B>;
    constexpr int PPP = B / 16;  // 1 KB pieces per part
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < R::NI; ++q) {
        const int piece = w + 4 * q;
        const int part = piece / PPP, pp = piece % PPP;
        const int pos = pp * 64 + lane;
        const int row = pos >> 2, kg = ((pos & 3) - bf16_rot(row)) & 3;
        // wave-uniform base plus the lane's 32-bit offset inside the part:
        // one VGPR per lane instead of a 64-bit address per piece, which
        // keeps the split-BF16 kernels within their registers (no spills)
        const char* base = blk + (size_t)part * B * B * 2 + chunk * 64;
        const uint32_t lofs = (uint32_t)(row * B * 2 + kg * 16);
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(base + lofs),
                                         (__attribute__((address_space(3))) void*)(lds_dst + piece * 1024), 16, 0,
                                         0);
    }
}

// Read-only (for the whole launch) data at a wave-uniform index, through the
// constant address space: a scalar load, which never waits behind vector
// memory operations in flight.
SPAMM_DEV int32_t const_ld(const int32_t* p, int idx) {
    const __attribute__((address_space(4))) int32_t* q = (const __attribute__((address_space(4))) int32_t*)(uintptr_t)p;
    return q[idx];
}
SPAMM_DEV int2 const_ld(const int2* p, int idx) {
    const __attribute__((address_space(4))) int64_t* q = (const __attribute__((address_space(4))) int64_t*)(uintptr_t)p;
    const int64_t v = q[idx];
    return make_int2((int32_t)(v & 0xffffffff), (int32_t)(v >> 32));
}

// 32-bit LDS address of a pointer into LDS
SPAMM_DEV uint32_t lds_addr(const char* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char*)p;
}

// The FP64 operand reads of one k-step: T doubles of A at a, a + 128, ...
// and T of B at b, b + 128, ... (byte addresses in LDS), waited for inside
// the same block.  Written out so that the compiler's memory model does not
// see LDS reads here: it cannot tell which ring slot the copies in flight
// fill once they cross the stage loop's back edge, and would drain every
// copy before the first read of each loop iteration.  The stage's own
// vmcnt wait and barrier order these reads after the copies of their slot,
// and the barrier of the next stage orders them before the slot's refill.
template <int T>
SPAMM_DEV void lds_read_tiles(uint32_t a, uint32_t b, double* av, double* bv);

template <>
SPAMM_DEV void lds_read_tiles<1>(uint32_t a, uint32_t b, double* av, double* bv) {
    double x, y;
    asm volatile("ds_read_b64 %0, %2\n\tds_read_b64 %1, %3\n\ts_waitcnt lgkmcnt(0)"
                 : "=&v"(x), "=&v"(y)
                 : "v"(a), "v"(b));
    av[0] = x;
    bv[0] = y;
}

template <>
SPAMM_DEV void lds_read_tiles<2>(uint32_t a, uint32_t b, double* av, double* bv) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 x, y;
    asm volatile("ds_read2_b64 %0, %2 offset1:16\n\tds_read2_b64 %1, %3 offset1:16\n\ts_waitcnt lgkmcnt(0)"
                 : "=&v"(x), "=&v"(y)
                 : "v"(a), "v"(b));
    av[0] = x[0];
    av[1] = x[1];
    bv[0] = y[0];
    bv[1] = y[1];
}

template <>
SPAMM_DEV void lds_read_tiles<4>(uint32_t a, uint32_t b, double* av, double* bv) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 x0, x1, y0, y1;
    asm volatile(
        "ds_read2_b64 %0, %4 offset1:16\n\tds_read2_b64 %1, %4 offset0:32 offset1:48\n\t"
        "ds_read2_b64 %2, %5 offset1:16\n\tds_read2_b64 %3, %5 offset0:32 offset1:48\n\ts_waitcnt lgkmcnt(0)"
        : "=&v"(x0), "=&v"(x1), "=&v"(y0), "=&v"(y1)
        : "v"(a), "v"(b));
    av[0] = x0[0];
    av[1] = x0[1];
    av[2] = x1[0];
    av[3] = x1[1];
    bv[0] = y0[0];
    bv[1] = y0[1];
    bv[2] = y1[0];
    bv[3] = y1[1];
}

// One LDS object per ring slot, and the stage loop unrolled by NS so every
// access names its slot statically: the compiler can then see that the
// copies in flight (other slots) never alias the slot being read, and only
// the explicit vmcnt waits order them.
template <int B, int S>
struct RingSlot {
    static SPAMM_DEV char* get() {
        __shared__ __attribute__((aligned(1024))) char mem[RingCfg<B>::STAGE];
        return mem;
    }
};

// Schedule of the ring kernels: workgroups per CU of the persistent grid, by
// leaf size (32, 64, 128).  Defaults: as many as the register and LDS
// budgets keep resident; settable (the autotuner measures the choices).
static int g_ring_per_cu[3] = {4, 3, 2};

static int leaf_index(int b) { return b == 32 ? 0 : (b == 64 ? 1 : 2); }

int get_ring_per_cu(int b) { return g_ring_per_cu[leaf_index(b)]; }
void set_ring_per_cu(int b, int per_cu) { g_ring_per_cu[leaf_index(b)] = per_cu; }

// persistent grid: a multiple of 8 so every XCD gets the same count
inline int ring_grid(int b, int num_cu) {
    const int per_cu = get_ring_per_cu(b);
    return (num_cu * per_cu + 7) / 8 * 8;
}

template <int B, int LOWT>
struct RingCtx {
    using R = RingCfg<B>;
    // operands of the current output (wave-uniform)
    const int2* pairs;
    const double* valA;
    const double* valB;
    const float* valA32;
    const float* valB32;
    const uint16_t* valA16;
    const uint16_t* valB16;
    const int32_t* expA;
    const int32_t* expB;
    int p0, nlow, nst_low, nst;
    d4 acc[R::TM][R::TN];
    f4 acc32[R::TM][R::TN];

    SPAMM_DEV void bind(const GemmArgs& g) {
        pairs = g.pairs;
        valA = g.valA;
        valB = g.valB;
        valA32 = g.valA32;
        valB32 = g.valB32;
        valA16 = g.valA16;
        valB16 = g.valB16;
        expA = g.expA;
        expB = g.expB;
    }

    template <int SLOT>
    SPAMM_DEV void issue(int st) {
        char* dst = RingSlot<B, SLOT>::get();
        int pr_i, chunk;
        bool low;
        if (LOWT && st < nst_low) {
            pr_i = st / R::CH32; chunk = st % R::CH32; low = true;
        } else {
            const int s2 = st - nst_low;
            pr_i = nlow + s2 / R::CH64; chunk = s2 % R::CH64; low = false;
        }
        // the pair list is read-only during the launch: read it through the
        // constant address space (scalar loads, counted apart from the copies)
        const int2 pr = const_ld(pairs, p0 + pr_i);
        if constexpr (LOWT == 2) {
            if (low) {
                dma_bf16_chunk<B>(reinterpret_cast<const char*>(valA16 + (size_t)pr.x * 2 * B * B), chunk, dst);
                dma_bf16_chunk<B>(reinterpret_cast<const char*>(valB16 + (size_t)pr.y * 2 * B * B), chunk,
                                  dst + R::OPB);
                return;
            }
        }
        const char* a0;
        const char* b0;
        const bool f64 = !(LOWT == 1 && low);
        if (LOWT == 1 && low) {
            a0 = reinterpret_cast<const char*>(valA32 + (size_t)pr.x * B * B + (size_t)chunk * R::KC32 * B);
            b0 = reinterpret_cast<const char*>(valB32 + (size_t)pr.y * B * B + (size_t)chunk * R::KC32 * B);
        } else if (pr.x >= 0) {
            a0 = reinterpret_cast<const char*>(valA + (size_t)pr.x * B * B + (size_t)chunk * R::KC64 * B);
            b0 = reinterpret_cast<const char*>(valB + (size_t)pr.y * B * B + (size_t)chunk * R::KC64 * B);
        } else {
            // a pair of the second kind (one's complement first slot): the
            // first operand comes from the B pool, the second from the A pool
            a0 = reinterpret_cast<const char*>(valB + (size_t)(~pr.x) * B * B + (size_t)chunk * R::KC64 * B);
            b0 = reinterpret_cast<const char*>(valA + (size_t)pr.y * B * B + (size_t)chunk * R::KC64 * B);
        }
        if constexpr (B == 32) {
            if (f64) {
                dma_chunk_rot<B>(a0, dst);
                dma_chunk_rot<B>(b0, dst + R::OPB);
                return;
            }
        }
        dma_chunk<B>(a0, dst);
        dma_chunk<B>(b0, dst + R::OPB);
    }

    template <int SLOT>
    SPAMM_DEV void compute(int st) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int wm = w >> 1, wn = w & 1;
        const char* sl = RingSlot<B, SLOT>::get();
        if (LOWT == 2 && st < nst_low) {
            // split-BF16 stage: 32 inner indices, parts hi and lo of A and B
            // (rotated rows of four 16 B groups, see bf16_rot); the A
            // rows go in the order pi(m) = m/4 + 4(m%4) as in the FP32 tier
            const int mrow = ((lane & 15) >> 2) + 4 * (lane & 3);
            const int kg = lane >> 4;
            auto rd = [&](const char* part, int row) -> bf8 {
                const int pos = row * 4 + ((kg + bf16_rot(row)) & 3);
                return *reinterpret_cast<const bf8*>(part + pos * 16);
            };
            const char* Ah = sl;
            const char* Al = sl + B * 64;
            const char* Bh = sl + R::OPB;
            const char* Bl = sl + R::OPB + B * 64;
            bf8 ah[R::TM], al[R::TM], bh[R::TN], bl[R::TN];
#pragma unroll
            for (int a = 0; a < R::TM; ++a) {
                ah[a] = rd(Ah, wm * R::TM * 16 + a * 16 + mrow);
                al[a] = rd(Al, wm * R::TM * 16 + a * 16 + mrow);
            }
#pragma unroll
            for (int b = 0; b < R::TN; ++b) {
                bh[b] = rd(Bh, wn * R::TN * 16 + b * 16 + (lane & 15));
                bl[b] = rd(Bl, wn * R::TN * 16 + b * 16 + (lane & 15));
            }
#pragma unroll
            for (int a = 0; a < R::TM; ++a)
#pragma unroll
                for (int b = 0; b < R::TN; ++b) {
                    acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc32[a][b], 0, 0, 0);
                    acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc32[a][b], 0, 0, 0);
                    acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc32[a][b], 0, 0, 0);
                }
            if ((st % R::CH32) == R::CH32 - 1) {
                // end of one pair: undo the two blocks' scalings (exact) and
                // fold into FP64
                const int2 pr = const_ld(pairs, p0 + st / R::CH32);
                const int e = const_ld(expA, pr.x) + const_ld(expB, pr.y);
#pragma unroll
                for (int a = 0; a < R::TM; ++a)
#pragma unroll
                    for (int b = 0; b < R::TN; ++b) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[a][b][r] = acc[a][b][r] + ldexp((double)acc32[a][b][r], e);
                        acc32[a][b] = f4{0.f, 0.f, 0.f, 0.f};
                    }
            }
        } else if (LOWT == 1 && st < nst_low) {
            const float* As = reinterpret_cast<const float*>(sl);
            const float* Bs = reinterpret_cast<const float*>(sl + R::OPB);
            // The f32 16x16x4 result puts row 4(l>>4)+r in register r of lane
            // l; the f64 one puts row (l>>4)+4r there.  Feeding the f32 MFMA
            // the A rows in the order pi(m) = m/4 + 4(m%4) makes both results
            // share one layout, so a finished FP32 pair product adds straight
            // into the FP64 accumulator.
            const int mrow = ((lane & 15) >> 2) + 4 * (lane & 3);
            // rows of the FP32 copies are rotated (f32_rot) so that the four
            // k rows one read touches fall in different banks
            const int rot = f32_rot<B>(lane >> 4);
#pragma unroll
            for (int ks = 0; ks < R::KC32 / 4; ++ks) {
                const int kr = ks * 4 + (lane >> 4);
                float av[R::TM], bv[R::TN];
#pragma unroll
                for (int a = 0; a < R::TM; ++a)
                    av[a] = As[kr * B + ((wm * R::TM * 16 + a * 16 + mrow + rot) & (B - 1))];
#pragma unroll
                for (int b = 0; b < R::TN; ++b)
                    bv[b] = Bs[kr * B + ((wn * R::TN * 16 + b * 16 + (lane & 15) + rot) & (B - 1))];
#pragma unroll
                for (int a = 0; a < R::TM; ++a)
#pragma unroll
                    for (int b = 0; b < R::TN; ++b)
                        acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc32[a][b], 0, 0, 0);
            }
            if ((st % R::CH32) == R::CH32 - 1) {
                // end of one low-tier pair: fold its FP32 product into FP64
#pragma unroll
                for (int a = 0; a < R::TM; ++a)
#pragma unroll
                    for (int b = 0; b < R::TN; ++b) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[a][b][r] = acc[a][b][r] + (double)acc32[a][b][r];
                        acc32[a][b] = f4{0.f, 0.f, 0.f, 0.f};
                    }
            }
        } else {
            // LDS byte addresses of this lane's first A and B element
            const uint32_t lbase = lds_addr(sl);
            // (leaf 32: rows rotated by f64_rot32; k = 4 ks + (lane >> 4) has the parity of lane >> 4)
            const int rot = B == 32 ? f64_rot32(lane >> 4) : 0;
            const uint32_t a0 =
                lbase + 8u * (uint32_t)((lane >> 4) * B + ((wm * R::TM * 16 + (lane & 15) + rot) & (B - 1)));
            const uint32_t b0 =
                lbase + R::OPB + 8u * (uint32_t)((lane >> 4) * B + ((wn * R::TN * 16 + (lane & 15) + rot) & (B - 1)));
            auto kstep = [&](int ks) {
                double av[R::TM], bv[R::TN];
                lds_read_tiles<R::TM>(a0 + (uint32_t)(ks * 4 * B * 8), b0 + (uint32_t)(ks * 4 * B * 8), av, bv);
#pragma unroll
                for (int a = 0; a < R::TM; ++a)
#pragma unroll
                    for (int b = 0; b < R::TN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
            };
            if constexpr (LOWT == 0) {
#pragma unroll
                for (int ks = 0; ks < R::KC64 / 4; ++ks) kstep(ks);
            } else {
                // the tier kernels unroll the FP64 stages by two so that their
                // registers fit three waves per SIMD
#pragma unroll 2
                for (int ks = 0; ks < R::KC64 / 4; ++ks) kstep(ks);
            }
        }
    }

    // one pipeline step on ring slot SLOT (stage st): wait for this stage,
    // barrier, refill the slot freed by the previous step, multiply
    template <int SLOT>
    SPAMM_DEV void step(int st) {
        const int ahead = min(R::NS - 2, nst - 1 - st);
        if (ahead >= 2) wait_vmcnt<2 * 2 * R::NI>();
        else if (ahead == 1) wait_vmcnt<2 * R::NI>();
        else wait_vmcnt<0>();
        __builtin_amdgcn_s_barrier();
        if (st + R::NS - 1 < nst) issue<(SLOT + R::NS - 1) % R::NS>(st + R::NS - 1);
        compute<SLOT>(st);
    }
};

// One output block (i, j) on the ring, in three parts so that the next
// output's first copies overlap this output's epilogue:
//   ring_begin     binds pairs p0 .. p1 (the first nlow low-tier) and issues
//                  the first NS - 1 stages into ring slots 0 .. NS - 2;
//   ring_multiply  runs every stage; returns with nothing in flight and all
//                  waves past their last read of the ring;
//   ring_epilogue  writes the block (and its mirror) through ring slot NS - 1
//                  used as a tile of EPC columns: the combine 2X - C when beta,
//                  and their norm when asked for.
template <int B, int LOWT>
SPAMM_DEV void ring_begin(RingCtx<B, LOWT>& cx, int p0, int p1, int nlow) {
    using R = RingCfg<B>;
    cx.p0 = p0;
    cx.nlow = LOWT ? nlow : 0;
    cx.nst_low = cx.nlow * R::CH32;
    cx.nst = cx.nst_low + (p1 - p0 - cx.nlow) * R::CH64;
    const int nst = cx.nst;
    if (0 < nst) cx.template issue<0>(0);
    if (R::NS > 2 && 1 < nst) cx.template issue<1 % R::NS>(1);
    if (R::NS > 3 && 2 < nst) cx.template issue<2 % R::NS>(2);
}

template <int B, int LOWT>
SPAMM_DEV void ring_multiply(RingCtx<B, LOWT>& cx) {
    using R = RingCfg<B>;
#pragma unroll
    for (int a = 0; a < R::TM; ++a)
#pragma unroll
        for (int b = 0; b < R::TN; ++b) {
            cx.acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
            if constexpr (LOWT != 0) cx.acc32[a][b] = f4{0.f, 0.f, 0.f, 0.f};
        }
    const int nst = cx.nst;
    for (int st = 0; st < nst; st += R::NS) {
        cx.template step<0>(st);
        if (st + 1 < nst) cx.template step<1 % R::NS>(st + 1);
        if (R::NS > 2 && st + 2 < nst) cx.template step<2 % R::NS>(st + 2);
        if (R::NS > 3 && st + 3 < nst) cx.template step<3 % R::NS>(st + 3);
    }
    wait_vmcnt<0>();
    __syncthreads();
}

// Norm of the block just written (and of its mirror, the same sum): the
// four waves' double-double partial sums (a, with the flags fl_w: 1 special,
// 2 tiny) are added in wave order; certified
// results are stored, the rest listed for the norms kernel.  The partials'
// LDS is next written in the following output's epilogue, after barriers
// that thread 0 reaches only when done reading.
SPAMM_DEV void block_norm_out(dd a, int fl_w, const GemmArgs& d, int sh, int sht) {
    __shared__ double s_part[4][2];
    __shared__ int s_flag[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (lane == 0) {
        s_part[w][0] = a.hi;
        s_part[w][1] = a.lo;
        s_flag[w] = fl_w;
    }
    __syncthreads();
    if (tid == 0) {
        dd t = {s_part[0][0], s_part[0][1]};
        int fl = s_flag[0];
        for (int q = 1; q < 4; ++q) {
            t = dd_add(t, dd{s_part[q][0], s_part[q][1]});
            fl |= s_flag[q];
        }
        if (sq_certified(t, fl & 1, fl & 2)) {
            const double nv = sqrt(t.hi);
            d.sq_out[sh] = t.hi;
            d.sqlo_out[sh] = t.lo;
            d.nrm_out[sh] = nv;
            if (sht >= 0) {
                d.sq_out[sht] = t.hi;
                d.sqlo_out[sht] = t.lo;
                d.nrm_out[sht] = nv;
            }
        } else {
            const int q = atomicAdd(d.nrecheck, sht >= 0 ? 2 : 1);
            d.recheck[q] = sh;
            if (sht >= 0) d.recheck[q + 1] = sht;
        }
    }
}

template <int B, int LOWT>
SPAMM_DEV void ring_epilogue(RingCtx<B, LOWT>& cx, const GemmArgs& d, int i, int j, bool beta) {
    using R = RingCfg<B>;
    constexpr int PC = 16;  // epilogue columns per pass
    static_assert(PC * R::LDT * 8 <= R::STAGE && B % PC == 0, "epilogue tile fits one ring slot");
    double* ldsd = reinterpret_cast<double*>(RingSlot<B, R::NS - 1>::get());
    // the thread index passes through an empty asm so that the epilogue's
    // per-lane addresses are formed here, per output, rather than hoisted
    // out of the persistent loop: the tier kernels then need no scratch
    // (a spilled address's reload waits for every copy in flight)
    int tid = threadIdx.x;
    if constexpr (LOWT != 0) asm volatile("" : "+v"(tid));
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int sh = d.map_out[(size_t)i * d.nb + j];
    const int sht = (d.sym && i != j) ? d.map_out[(size_t)j * d.nb + i] : -1;
    const int sx = beta ? d.mapX[(size_t)i * d.nb + j] : -1;
    double* dst = sh >= 0 ? d.val_out + (size_t)sh * B * B : nullptr;
    double* dstt = sht >= 0 ? d.val_out + (size_t)sht * B * B : nullptr;
    const double* xs = sx >= 0 ? d.valX + (size_t)sx * B * B : nullptr;
    const bool want_norm = d.sq_out && dst;
    // the FP32-tier kernels also write the blocks' FP32 copies for the next step
    float* d32 = (LOWT == 1 && d.out32 && sh >= 0) ? d.out32 + (size_t)sh * B * B : nullptr;
    float* d32t = (LOWT == 1 && d.out32 && sht >= 0) ? d.out32 + (size_t)sht * B * B : nullptr;
    // each lane's share of the block's sum of squares; in the tier kernels
    // at leaf 64, whose registers are scarce, its running total waits in
    // ring slot NS - 1 behind the epilogue tile between passes
    constexpr bool kLdsSum = LOWT != 0 && B == 64;
    constexpr int kSumOff = (PC * R::LDT * 8 + 15) / 16 * 16;
    static_assert(!kLdsSum || kSumOff + 256 * 16 <= R::STAGE, "partial sums fit the ring slot");
    dd* lsum = reinterpret_cast<dd*>(reinterpret_cast<char*>(ldsd) + kSumOff);
    SqAcc sa;
    for (int pass = 0; pass < B / PC; ++pass) {
        if (kLdsSum) sa.acc = dd{0.0, 0.0};
        const int c0 = pass * PC;
#pragma unroll
        for (int a = 0; a < R::TM; ++a)
#pragma unroll
            for (int b = 0; b < R::TN; ++b) {
                const int col = wn * R::TN * 16 + b * 16 + (lane & 15);
                if (col < c0 || col >= c0 + PC) continue;
                const int rowb = wm * R::TM * 16 + a * 16 + (lane >> 4);
#pragma unroll
                for (int r = 0; r < 4; ++r) ldsd[(col - c0) * R::LDT + rowb + 4 * r] = cx.acc[a][b][r];
            }
        __syncthreads();
        for (int e = tid; e < PC * B; e += 256) {
            const int cl = e / B, row = e % B;
            double v = ldsd[cl * R::LDT + row];
            if (beta) {
                const double x = xs ? xs[(size_t)(c0 + cl) * B + row] : 0.0;
                v = 2.0 * x - v;
                ldsd[cl * R::LDT + row] = v;
            }
            if (dst) dst[(size_t)(c0 + cl) * B + row] = v;
            if (want_norm) sq_add(sa, v);
            if (LOWT == 1 && d32) d32[(c0 + cl) * B + ((row + f32_rot<B>(c0 + cl)) & (B - 1))] = (float)v;
        }
        if (dstt) {
            __syncthreads();
            for (int e = tid; e < PC * B; e += 256) {
                const int cp = e / PC, rp = e % PC;
                const double v = ldsd[rp * R::LDT + cp];
                dstt[(size_t)cp * B + c0 + rp] = v;
                if (LOWT == 1 && d32t) d32t[cp * B + ((c0 + rp + f32_rot<B>(cp)) & (B - 1))] = (float)v;
            }
        }
        if (kLdsSum && want_norm) lsum[tid] = pass ? dd_add(lsum[tid], sa.acc) : sa.acc;  // own entry
        __syncthreads();
    }
    if (want_norm) {
        if (kLdsSum) sa.acc = lsum[tid];
        const int fl = (__any(sa.special) ? 1 : 0) | (__any(sa.tiny) ? 2 : 0);
        block_norm_out(dd_wave_sum(sa.acc), fl, d, sh, sht);
    }
}

// First output of XCD range xcd (0..8): outputs are cut where the running
// pair count first reaches np * xcd / 8; pair_before(o) = pairs of the
// outputs before o (monotone, pair_before(nout) = np).
template <typename PB>
SPAMM_DEV int64_t xcd_cut(int64_t nout, int64_t np, int xcd, PB&& pair_before) {
    if (xcd >= 8) return nout;
    const int64_t t = np * xcd / 8;
    int64_t lo = 0, hi = nout;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (pair_before(mid) < t) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <int B, int LOWT>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(RingCfg<B>::template waves<LOWT>(), 8))) void k_gemm_ring(GemmArgs g) {
    using R = RingCfg<B>;
    static_assert(R::NS >= 2 && R::NS <= 4, "ring depth");
    __shared__ int s_o, s_cut[9];
    if (g.done && *g.done) return;
    if (g.ovf && *g.ovf) return;
    const int tid = threadIdx.x;
    const int64_t nout = *g.nout;
    // a grid larger than the output list: the first max(nout, 8) workgroups
    // (every XCD keeps one) claim every output, the rest leave at once
    if ((int64_t)blockIdx.x >= nout && blockIdx.x >= 8) return;
    const int xcd = blockIdx.x % 8;
    if (tid < 9) {
        if (g.cuts) {
            s_cut[tid] = g.cuts[tid];
        } else {
            const int64_t np = g.optr[nout];
            auto pb = [&](int64_t o) -> int64_t { return g.optr[o]; };
            s_cut[tid] = (int)xcd_cut(nout, np, tid, pb);
        }
    }
    __syncthreads();
    const bool beta = g.mapX && g.branch && (*g.branch == 1);
    RingCtx<B, LOWT> cx;
    cx.bind(g);
    // next output (wave-uniform, in scalar registers, so the pair list is
    // read with scalar loads that never wait behind the copies in flight):
    // from this XCD's range while it lasts, then from the other ranges in
    // turn, so that no XCD idles while another still has outputs; -1 once
    // every range is drained (at most 8 failed claims per workgroup, and none on
    // another range whose counter already shows it drained)
    int r = 0;
    auto fetch = [&]() -> int {
        if (tid == 0) {
            int on = -1;
            for (; r < 8; ++r) {
                const int x = (xcd + r) & 7;
                // another XCD's range: skip it when a plain load shows it
                // drained, so that with few outputs the many idle workgroups
                // do not queue atomics (serialised per counter) on empty
                // ranges; the own range is claimed at once (the load would
                // add its latency to every claim)
                if (r > 0 && __hip_atomic_load(&g.counters[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                                 s_cut[x + 1] - s_cut[x])
                    continue;
                const int c = s_cut[x] + atomicAdd(&g.counters[x], 1);
                if (c < s_cut[x + 1]) {
                    on = c;
                    break;
                }
            }
            s_o = on;
        }
        __syncthreads();
        const int o = __builtin_amdgcn_readfirstlane(s_o);
        __syncthreads();
        return o;
    };
    int o = fetch();
    if (o < 0) return;
    int i = const_ld(g.oi, o), j = const_ld(g.oj, o);
    ring_begin<B, LOWT>(cx, const_ld(g.optr, o), const_ld(g.optr, o + 1), LOWT ? const_ld(g.olow, o) : 0);
    while (true) {
        ring_multiply<B, LOWT>(cx);
        const int on = fetch();
        int in = 0, jn = 0;
        if (on >= 0) {
            in = const_ld(g.oi, on);
            jn = const_ld(g.oj, on);
            ring_begin<B, LOWT>(cx, const_ld(g.optr, on), const_ld(g.optr, on + 1), LOWT ? const_ld(g.olow, on) : 0);
        }
        ring_epilogue<B, LOWT>(cx, g, i, j, beta);
        wait_vmcnt<0>();  // the epilogue's accesses and the next output's first copies
        if (on < 0) break;
        i = in;
        j = jn;
    }
}

// Several independent products in one persistent launch: system s owns the
// global outputs out_off[s] .. out_off[s+1] and the pairs pair_off[s] ..
// pair_off[s+1] (exclusive prefix sums over the systems, k_batch_prefix);
// descs[s] holds its matrices and lists.
template <int B, int LOWT>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(RingCfg<B>::template waves<LOWT>(), 8))) void k_gemm_ring_batch(
    const GemmArgs* __restrict__ descs, int nsys, const int64_t* __restrict__ out_off,
    const int64_t* __restrict__ pair_off, int32_t* __restrict__ counters) {
    __shared__ int s_o, s_cut[9];
    const int tid = threadIdx.x;
    const int64_t nout = out_off[nsys];
    if ((int64_t)blockIdx.x >= nout && blockIdx.x >= 8) return;  // as in k_gemm_ring
    const int xcd = blockIdx.x % 8;
    auto sys_of = [&](int64_t o) -> int {
        int a = 0, z = nsys - 1;  // last s with out_off[s] <= o
        while (a < z) {
            const int m = (a + z + 1) >> 1;
            if (out_off[m] <= o) a = m; else z = m - 1;
        }
        return a;
    };
    if (tid < 9) {
        const int64_t np = pair_off[nsys];
        auto pb = [&](int64_t o) -> int64_t {
            if (o >= nout) return np;
            const int sy = sys_of(o);
            return pair_off[sy] + descs[sy].optr[o - out_off[sy]];
        };
        s_cut[tid] = (int)xcd_cut(nout, np, tid, pb);
    }
    __syncthreads();
    RingCtx<B, LOWT> cx;
    // next output: this XCD's range first, then the other ranges (as in
    // k_gemm_ring); -1 once all are drained
    int r = 0;
    auto fetch = [&]() -> int {
        if (tid == 0) {
            int on = -1;
            for (; r < 8; ++r) {
                const int x = (xcd + r) & 7;
                if (r > 0 && __hip_atomic_load(&counters[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                                 s_cut[x + 1] - s_cut[x])
                    continue;  // another range, drained (a plain load; see k_gemm_ring)
                const int c = s_cut[x] + atomicAdd(&counters[x], 1);
                if (c < s_cut[x + 1]) {
                    on = c;
                    break;
                }
            }
            s_o = on;
        }
        __syncthreads();
        const int o = __builtin_amdgcn_readfirstlane(s_o);
        __syncthreads();
        return o;
    };
    // bind output o (its system's descriptor) and issue its first stages
    auto begin = [&](int o, const GemmArgs*& dp, int& i, int& j) {
        const int sy = __builtin_amdgcn_readfirstlane(sys_of(o));
        dp = &descs[sy];
        const GemmArgs& d = *dp;
        const int ol = o - (int)out_off[sy];
        i = const_ld(d.oi, ol);
        j = const_ld(d.oj, ol);
        cx.bind(d);
        ring_begin<B, LOWT>(cx, const_ld(d.optr, ol), const_ld(d.optr, ol + 1), LOWT ? const_ld(d.olow, ol) : 0);
    };
    int o = fetch();
    if (o < 0) return;
    const GemmArgs* dc = nullptr;
    int i = 0, j = 0;
    begin(o, dc, i, j);
    while (true) {
        ring_multiply<B, LOWT>(cx);
        const int on = fetch();
        const GemmArgs* dn = nullptr;
        int in = 0, jn = 0;
        if (on >= 0) begin(on, dn, in, jn);
        const bool beta = dc->mapX && dc->branch && (*dc->branch == 1);
        ring_epilogue<B, LOWT>(cx, *dc, i, j, beta);
        wait_vmcnt<0>();  // the epilogue's accesses and the next output's first copies
        if (on < 0) break;
        dc = dn;
        i = in;
        j = jn;
    }
}

// out_off / pair_off over the systems whose step runs (not done, no overflow)
__global__ void k_batch_prefix(const GemmArgs* __restrict__ descs, int nsys, int64_t* __restrict__ out_off,
                               int64_t* __restrict__ pair_off) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t ao = 0, ap = 0;
    for (int s = 0; s < nsys; ++s) {
        out_off[s] = ao;
        pair_off[s] = ap;
        const GemmArgs& d = descs[s];
        const bool skip = (d.done && *d.done) || (d.ovf && *d.ovf);
        if (!skip) {
            const int64_t n = *d.nout;
            ao += n;
            ap += d.optr[n];
        }
    }
    out_off[nsys] = ao;
    pair_off[nsys] = ap;
}

__global__ void k_reset_counters(int32_t* c) {
    if (threadIdx.x < 16) c[threadIdx.x] = 0;
}

void launch_gemm_f64(const GemmArgs& g, int num_cu, hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_end,
                     bool counters_clear) {
    if (!counters_clear) hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, g.counters);
    if (ev_start) (void)hipEventRecord(ev_start, s);
    const int per_cu = g.b == 128 ? 2 : 4;
    int grid = num_cu * per_cu;
    grid = (grid + 7) / 8 * 8;
    const bool low = g.valA32 != nullptr;
    const bool low16 = g.valA16 != nullptr;
#define SPAMM_G(B_, T_, L_) hipLaunchKernelGGL((k_gemm<B_, T_, L_>), dim3(grid), dim3(256), 0, s, g)
#define SPAMM_GB(T_)                                                     \
    switch (g.b) {                                                       \
        case 32: if (low) SPAMM_G(32, T_, 1); else SPAMM_G(32, T_, 0); break; \
        case 64: if (low) SPAMM_G(64, T_, 1); else SPAMM_G(64, T_, 0); break; \
        case 128: SPAMM_G(128, T_, 0); break; /* no FP32 tier at leaf 128 */ \
    }
    if (g.btrans) {
        const int gr = ring_grid(g.b, num_cu);
        switch (g.b) {
            case 32: if (low16) hipLaunchKernelGGL((k_gemm_ring<32, 2>), dim3(gr), dim3(256), 0, s, g);
                     else if (low) hipLaunchKernelGGL((k_gemm_ring<32, 1>), dim3(gr), dim3(256), 0, s, g);
                     else hipLaunchKernelGGL((k_gemm_ring<32, 0>), dim3(gr), dim3(256), 0, s, g); break;
            case 64: if (low16) hipLaunchKernelGGL((k_gemm_ring<64, 2>), dim3(gr), dim3(256), 0, s, g);
                     else if (low) hipLaunchKernelGGL((k_gemm_ring<64, 1>), dim3(gr), dim3(256), 0, s, g);
                     else hipLaunchKernelGGL((k_gemm_ring<64, 0>), dim3(gr), dim3(256), 0, s, g); break;
            case 128: hipLaunchKernelGGL((k_gemm_ring<128, 0>), dim3(gr), dim3(256), 0, s, g); break;
        }
    } else {
        SPAMM_GB(false)
    }
    if (ev_end) (void)hipEventRecord(ev_end, s);
#undef SPAMM_GB
#undef SPAMM_G
}

void launch_gemm_batch(int b, int low, const GemmArgs* descs_dev, int nsys, int64_t* out_off, int64_t* pair_off,
                       int32_t* counters, int num_cu, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_prefix, dim3(1), dim3(64), 0, s, descs_dev, nsys, out_off, pair_off);
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, counters);
    const int gr = ring_grid(b, num_cu);
#define SPAMM_GBT(B_, L_)                                                                                       \
    hipLaunchKernelGGL((k_gemm_ring_batch<B_, L_>), dim3(gr), dim3(256), 0, s, descs_dev, nsys, out_off, pair_off, \
                       counters)
    switch (b) {
        case 32: if (low == 2) SPAMM_GBT(32, 2); else if (low) SPAMM_GBT(32, 1); else SPAMM_GBT(32, 0); break;
        case 64: if (low == 2) SPAMM_GBT(64, 2); else if (low) SPAMM_GBT(64, 1); else SPAMM_GBT(64, 0); break;
        case 128: SPAMM_GBT(128, 0); break;
    }
#undef SPAMM_GBT
}

// Round to the nearest BF16 value (8 significant bits, ties to even, BF16
// subnormal spacing 2^-133), in double arithmetic: every step is exact.
SPAMM_DEV double rn_bf16(double x) {
    if (x == 0.0) return x;
    int e;
    frexp(x, &e);
    int q = e - 8;
    if (q < -133) q = -133;
    return ldexp(rint(ldexp(x, -q)), q);
}

// bits of a BF16 value held exactly in a double
SPAMM_DEV uint16_t bf16_bits(double v) { return (uint16_t)(__float_as_uint((float)v) >> 16); }

// Split-BF16 copies of the live blocks: the block is scaled by 2^-e so that
// its largest |x| lies in [1, 2) (exact), then hi = RN_bf16(x'), lo =
// RN_bf16(x' - hi); both parts row-major, hi then lo per slot; expo = e.
// One workgroup per block: the threads read the column-major block with
// 16-byte loads (consecutive lanes, consecutive bytes) into an LDS copy with
// rows of B + 1 doubles, take the block's largest |x|, and then write both
// parts in 16-byte pieces of eight entries of a row, consecutive lanes
// writing consecutive pieces, so both the reads and the writes move whole
// lines.  The odd row stride keeps the column-order LDS writes and the
// row-order reads within two passes of the 64 banks at leaf 64.
template <int B>
__global__ __launch_bounds__(256) void k_to_bf16x2(const int32_t* __restrict__ nslot_p, int64_t cap,
                                                  const int32_t* __restrict__ brow, const double* __restrict__ val,
                                                  uint16_t* __restrict__ out, int32_t* __restrict__ expo,
                                                  const int32_t* __restrict__ done) {
    constexpr int LD = B + 1;          // LDS row stride in doubles
    constexpr int NV = B * B / 512;    // 16-byte loads per thread: 8 at leaf 64, 2 at leaf 32
    constexpr int NCH = B * B / 8;     // 16-byte pieces per part
    static_assert(NV >= 1 && B % 8 == 0, "leaf 32 or 64");
    __shared__ double tile[B * LD];
    __shared__ double s_m[4];
    if (done && *done) return;
    int64_t nslot = *nslot_p;
    if (nslot > cap) nslot = cap;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int64_t s = blockIdx.x; s < nslot; s += gridDim.x) {
        if (brow[s] < 0) continue;  // hole (workgroup-uniform)
        const double2* src = reinterpret_cast<const double2*>(val + (size_t)s * B * B);
        double2 v[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = src[q * 256 + t];
        double m = 0.0;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const int e = 2 * (q * 256 + t), c = e / B, r = e % B;  // column-major: entries (r, c), (r + 1, c)
            tile[r * LD + c] = v[q].x;
            tile[(r + 1) * LD + c] = v[q].y;
            m = fmax(m, fmax(fabs(v[q].x), fabs(v[q].y)));
        }
#pragma unroll
        for (int k = 32; k >= 1; k >>= 1) m = fmax(m, __shfl_xor(m, k));
        if (lane == 0) s_m[wv] = m;
        __syncthreads();
        m = fmax(fmax(s_m[0], s_m[1]), fmax(s_m[2], s_m[3]));
        int ex = 0;
        if (m > 0.0) frexp(m, &ex);
        const int sc = 1 - ex;  // x' = x 2^sc has its largest |x'| in [1, 2)
        uint4* hi = reinterpret_cast<uint4*>(out + (size_t)s * 2 * B * B);  // row-major destination
        uint4* lo = reinterpret_cast<uint4*>(out + (size_t)s * 2 * B * B + B * B);
        for (int j = t; j < NCH; j += 256) {
            const double* row = tile + (j / (B / 8)) * LD + 8 * (j % (B / 8));  // piece j: 8 entries of one row
            uint32_t hw[4], lw[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double x0 = ldexp(row[2 * q], sc), x1 = ldexp(row[2 * q + 1], sc);
                const double h0 = rn_bf16(x0), h1 = rn_bf16(x1);
                hw[q] = (uint32_t)bf16_bits(h0) | ((uint32_t)bf16_bits(h1) << 16);
                lw[q] = (uint32_t)bf16_bits(rn_bf16(x0 - h0)) | ((uint32_t)bf16_bits(rn_bf16(x1 - h1)) << 16);
            }
            hi[j] = uint4{hw[0], hw[1], hw[2], hw[3]};
            lo[j] = uint4{lw[0], lw[1], lw[2], lw[3]};
        }
        if (t == 0) expo[s] = -sc;
        __syncthreads();  // the next block rewrites the tile and s_m
    }
}

void launch_to_bf16x2(int b, const int32_t* nslot, int64_t cap, const int32_t* brow, const double* val, uint16_t* out,
                      int32_t* expo, const int32_t* done, hipStream_t s, int max_wg) {
    const int grid = grid_for(cap, 1, max_wg);
    switch (b) {
        case 32: hipLaunchKernelGGL((k_to_bf16x2<32>), dim3(grid), dim3(256), 0, s, nslot, cap, brow, val, out, expo, done); break;
        case 64: hipLaunchKernelGGL((k_to_bf16x2<64>), dim3(grid), dim3(256), 0, s, nslot, cap, brow, val, out, expo, done); break;
    }
}

// FP32 copies of the live blocks (round to nearest), for the low tier; with
// swz the rows (columns of the column-major block, index k) are rotated by
// f32_rot(k) for the ring kernel, else the copy keeps the block's layout.
template <int B>
__global__ __launch_bounds__(256) void k_to_f32(const int32_t* __restrict__ nslot_p, int64_t cap,
                                               const int32_t* __restrict__ brow, const double* __restrict__ val,
                                               float* __restrict__ out, int swz, const int32_t* __restrict__ done) {
    if (done && *done) return;
    int64_t nslot = *nslot_p;
    if (nslot > cap) nslot = cap;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t s = (int64_t)blockIdx.x * 4 + wv; s < nslot; s += (int64_t)gridDim.x * 4) {
        if (brow[s] < 0) continue;
        const double2* src = reinterpret_cast<const double2*>(val + (size_t)s * B * B);
        float2* dst = reinterpret_cast<float2*>(out + (size_t)s * B * B);
        // eight loads in flight per lane before their stores
        constexpr int IT = B * B / 128, U = IT < 8 ? IT : 8;
#pragma unroll 1
        for (int u0 = 0; u0 < IT; u0 += U) {
            double2 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = src[(u0 + u) * 64 + lane];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = (u0 + u) * 64 + lane;
                int d = t;
                if (swz) {
                    // element pair (m, m + 1) of row k, m even: stays a pair after the rotation
                    const int k = (2 * t) / B, m = (2 * t) % B;
                    d = (k * B + ((m + f32_rot<B>(k)) & (B - 1))) / 2;
                }
                dst[d] = float2{(float)v[u].x, (float)v[u].y};
            }
        }
    }
}

void launch_to_f32(int b, const int32_t* nslot, int64_t cap, const int32_t* brow, const double* val, float* out,
                   int swz, const int32_t* done, hipStream_t s) {
    const int grid = grid_for(cap, 4, 4096);
    switch (b) {
        case 32: hipLaunchKernelGGL(k_to_f32<32>, dim3(grid), dim3(256), 0, s, nslot, cap, brow, val, out, swz, done); break;
        case 64: hipLaunchKernelGGL(k_to_f32<64>, dim3(grid), dim3(256), 0, s, nslot, cap, brow, val, out, swz, done); break;
        case 128: hipLaunchKernelGGL(k_to_f32<128>, dim3(grid), dim3(256), 0, s, nslot, cap, brow, val, out, 0, done); break;
    }
}

}  // namespace spamm
