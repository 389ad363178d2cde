// gfx950 kernels and device entry points of the heffx library.
//
// bsgemm_f64: every GEMM of the sigma-vector path (operator mixing, the two
// rounds of block products, diag(H_eff), environment updates) is one launch of
// this kernel over a list of output tiles.  A tile (<= 64 x 64 of one output
// block) is owned by one workgroup, which sums alpha_j op(A_j) op(B_j) over its
// task list with the K dimensions of all tasks concatenated (no per-task
// padding) and writes the tile once: no atomics, fixed summation order, so FP64
// results are bitwise reproducible.  The inner product runs on the FP64 matrix
// cores (v_mfma_f64_16x16x4_f64); each of the 4 waves owns a 32 x 32 quadrant
// (2 x 2 MFMA tiles); K stages (16 or 8 deep) are staged through LDS (one or two
// buffers) with a register prefetch of the next stage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <cstdio>
#include <string>

#include "heffx.h"
#include "heffx_internal.h"

using namespace hx;

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));

// FP32 -> BF16 bit pattern, round to nearest even (v_cvt_pk_bf16_f32, low half).
// Each value is converted on its own: this compiler lowers a two-element vector
// conversion to one instruction that reads the first element twice.
__device__ __forceinline__ unsigned short to_bf16(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }

template <typename T>
struct BasesT {
    T* p[SP_N];
};
using Bases = BasesT<double>;

// Select a space's base pointer without indexing the argument array dynamically
// (which would move it to scratch).  NSP: number of spaces the launch can name
// (the sigma-vector and environment paths use the first 7, the adjoint all).
template <typename T, int NSP = SP_N>
__device__ __forceinline__ T* space_ptr(const BasesT<T>& B, int sp) {
    T* r = B.p[0];
#pragma unroll
    for (int i = 1; i < NSP; ++i) r = sp == i ? B.p[i] : r;
    return r;
}

constexpr int NSP_FWD = SP_PART + 1;

// The K range of a tile is walked in stages of KSV (16 or 8, the plan's variant);
// every task's K is padded to a multiple of KSV with zeros, so a stage belongs to
// exactly one task and the walk is uniform across the workgroup (scalar
// registers, one lookup per stage).

// Uniform task cursor of a tile.  The current task's operand bases are kept in
// scalar registers and the next task's descriptor is fetched one task ahead, so
// a K stage inside a task issues no scalar memory load before its vector loads.
template <typename T, bool TA, bool TB, int NSP, int KSV>
struct Cursor {
    int j, tend, kl;
    int lda, ldb, k;
    T alpha;
    const T* a;  // A at the tile origin, first k of the task
    const T* b;
    Task nxt;

    __device__ __forceinline__ void bind(const Task& t, const BasesT<T>& B, int r0, int c0) {
        lda = t.lda;
        ldb = t.ldb;
        k = t.k;
        alpha = (T)t.alpha;
        a = space_ptr<T, NSP>(B, t.spaces & 0xff) + t.aoff + (TA ? (int64_t)r0 : (int64_t)r0 * t.lda);
        b = space_ptr<T, NSP>(B, (t.spaces >> 8) & 0xff) + t.boff + (TB ? (int64_t)c0 * t.ldb : (int64_t)c0);
    }

    __device__ __forceinline__ void start(int tbeg, int tend_, const Task* __restrict__ tasks, const BasesT<T>& B,
                                          int r0, int c0) {
        j = tbeg;
        tend = tend_;
        kl = 0;
        k = 0;
        if (j < tend) bind(tasks[j], B, r0, c0);
        if (j + 1 < tend) nxt = tasks[j + 1];
    }

    // Position of the next K stage: operand pointers at its first k, valid depth krem.
    __device__ __forceinline__ void next(const Task* __restrict__ tasks, const BasesT<T>& B, int r0, int c0,
                                         const T*& pa, const T*& pb, int& krem, T& al) {
        while (j < tend && kl >= k) {
            ++j;
            kl = 0;
            if (j < tend) {
                bind(nxt, B, r0, c0);
                if (j + 1 < tend) nxt = tasks[j + 1];
            }
        }
        if (j >= tend) {
            pa = pb = nullptr;
            krem = 0;
            al = 0;
            return;
        }
        pa = a + (TA ? (int64_t)kl * lda : (int64_t)kl);
        pb = b + (TB ? (int64_t)kl : (int64_t)kl * ldb);
        krem = min(KSV, k - kl);
        al = alpha;
        kl += KSV;
    }
};

constexpr int LDS_PAD = 1;

// Element type T: double (v_mfma_f64_16x16x4_f64) or float (v_mfma_f32_16x16x4_f32,
// FP32 accumulation).  The tile tables are the same for both.
// KSV: K-stage depth (16 or 8); NBUF: LDS buffers (2: the next stage is stored
// while the current one is read; 1: half the LDS, one more barrier per stage).
// BF (T = float only): operands are rounded to BF16 at the LDS store and the
// products run on v_mfma_f32_16x16x16_bf16 with FP32 accumulation; LDS then holds
// each tile row's 16 k contiguously so a lane's 4 consecutive k are one 8-byte read.
// WR: waves stacked along the tile's rows (2: 64 x 64 tile, 4: 128 x 32, 1: 32 x 128);
// each wave owns a 32 x 32 quadrant.
template <typename T, bool TA, bool TB, int NSP, int KSV, int NBUF, bool BF = false, int WR = 2>
__global__ __launch_bounds__(256) void bsgemm(const Tile* __restrict__ tiles, const Task* __restrict__ tasks,
                                              BasesT<T> B, int ntile) {
    using acc_t = typename std::conditional<std::is_same<T, double>::value, dbl4, flt4>::type;
    static_assert(KSV == 8 || KSV == 16 || (KSV == 32 && std::is_same<T, float>::value), "stage depth");
    static_assert(!BF || (std::is_same<T, float>::value && KSV >= 16), "BF16 products: FP32 storage, 16-deep stages");
    static_assert(WR == 1 || WR == 2 || WR == 4, "wave layout");
    // KSV 32 (FP32 storage): a stage is two consecutive 16-deep K segments of the
    // plan (every task's K is padded to 16), each inside one task, possibly two tasks
    constexpr int KP = KSV == 32 ? 16 : KSV;  // K segment of the plan walked by the cursor
    constexpr int TMS = 32 * WR, TNS = 32 * (4 / WR);  // tile extent
    constexpr int NEA = TMS * KSV / 256;  // elements of A each thread stages per K stage
    constexpr int NEB = TNS * KSV / 256;  // ... and of B
    constexpr int LDB = KSV == 32 ? 40 : KSV + 4; // BF16 row pitch (8- / 16-byte aligned rows)
    __shared__ T As[BF ? 1 : NBUF][BF ? 1 : KSV][BF ? 1 : TMS + LDS_PAD];
    __shared__ T Bs[BF ? 1 : NBUF][BF ? 1 : KSV][BF ? 1 : TNS + LDS_PAD];
    __shared__ __attribute__((aligned(16))) unsigned short Ah[BF ? NBUF : 1][BF ? TMS : 1][BF ? LDB : 1];
    __shared__ __attribute__((aligned(16))) unsigned short Bh[BF ? NBUF : 1][BF ? TNS : 1][BF ? LDB : 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr0 = (wave % WR) * 32;
    const int wc0 = (wave / WR) * 32;
    // load lanes (element e of a thread: idx = tid + 256 e):
    //  A !TA: k = idx % KSV, row = idx / KSV (KSV contiguous k per row)
    //  A  TA: row = idx % TMS, k = idx / TMS (TMS contiguous rows per k)
    //  B !TB: col = idx % TNS, k = idx / TNS
    //  B  TB: k = idx % KSV, col = idx / KSV
    const int a_r = TA ? (tid % TMS) : (tid / KSV);
    const int a_k = TA ? (tid / TMS) : (tid % KSV);
    const int b_c = TB ? (tid / KSV) : (tid % TNS);
    const int b_k = TB ? (tid % KSV) : (tid / TNS);
    constexpr int a_dr = TA ? 0 : 256 / KSV, a_dk = TA ? 256 / TMS : 0;  // step per element e
    constexpr int b_dc = TB ? 256 / KSV : 0, b_dk = TB ? 0 : 256 / TNS;

    int t = blockIdx.x;
    Tile tl = tiles[t];
    acc_t acc00, acc01, acc10, acc11;
    T ra[NEA], rb[NEB];
    T alpha = 0;

    // Loader of the tile's K stages and the stage held in ra / rb.
    Cursor<T, TA, TB, NSP, KP> cur;
    int lm = 0, ln = 0, lr0 = 0, lc0 = 0;       // extent and origin of the loader's tile
    int krem_ld = 0, m_ld = 0, n_ld = 0;         // valid depth / extent of the held stage
    int krem_ld2 = 0;                            // KSV 32: valid depth of its second segment
    T alpha2 = 0;                                // ... and that segment's coefficient
    int kst0 = 0, kst1 = 0;                      // valid depth of the stage in LDS buffer 0 / 1
    int kst0b = 0;                               // KSV 32, one buffer: of its second segment
    auto bind_loader = [&](const Tile& x) {
        lm = x.m;
        ln = x.n;
        lr0 = x.r0;
        lc0 = x.c0;
        cur.start(x.tbeg, x.tend, tasks, B, lr0, lc0);
    };
    // Every K stage of a tile lies inside one task (krem >= 1), so indices clamped to
    // the block are always valid addresses: the FP32 loads issue unconditionally and
    // stay in flight across the MFMA work; elements outside the block are zeroed at
    // the LDS store (A through its 0/alpha factor).  FP64 (measured faster this way)
    // loads under exec masks, so padding rows and columns issue no memory requests.
    // Offsets inside one block fit in 32 bits.
    auto load_stage = [&]() {
        const T *qa, *qb;
        int krem;
        cur.next(tasks, B, lr0, lc0, qa, qb, krem, alpha);
        const int lda = cur.lda, ldb = cur.ldb;
        // KSV 32: the second segment (qa2, qb2; lda2, ldb2); without one (the tile's
        // last stage), the first segment's addresses stand in and are zeroed at the store
        const T *qa2 = qa, *qb2 = qb;
        int krem2 = 0, lda2 = lda, ldb2 = ldb;
        if constexpr (KSV == 32) {
            const T *pa, *pb;
            T al;
            cur.next(tasks, B, lr0, lc0, pa, pb, krem2, al);
            if (krem2 > 0) {
                qa2 = pa;
                qb2 = pb;
                lda2 = cur.lda;
                ldb2 = cur.ldb;
                alpha2 = al;
            }
        }
#pragma unroll
        for (int e = 0; e < NEA; ++e) {
            const int r = a_r + a_dr * e, ka = a_k + a_dk * e;
            if constexpr (std::is_same<T, double>::value) {
                T va = 0;
                if (ka < krem && r < lm) va = qa[TA ? ka * lda + r : r * lda + ka];
                ra[e] = va;
            } else if constexpr (KSV == 32) {
                const bool h = ka >= KP;  // the element's segment
                const int kk = ka & (KP - 1), kr = h ? krem2 : krem, ld = h ? lda2 : lda;
                const T* q = h ? qa2 : qa;
                const int rc = min(r, lm - 1), kac = max(min(kk, kr - 1), 0);
                ra[e] = q[TA ? kac * ld + rc : rc * ld + kac];
            } else {
                const int rc = min(r, lm - 1), kac = min(ka, krem - 1);
                ra[e] = qa[TA ? kac * lda + rc : rc * lda + kac];
            }
        }
#pragma unroll
        for (int e = 0; e < NEB; ++e) {
            const int c = b_c + b_dc * e, kb = b_k + b_dk * e;
            if constexpr (std::is_same<T, double>::value) {
                T vb = 0;
                if (kb < krem && c < ln) vb = qb[TB ? c * ldb + kb : kb * ldb + c];
                rb[e] = vb;
            } else if constexpr (KSV == 32) {
                const bool h = kb >= KP;
                const int kk = kb & (KP - 1), kr = h ? krem2 : krem, ld = h ? ldb2 : ldb;
                const T* q = h ? qb2 : qb;
                const int cc = min(c, ln - 1), kbc = max(min(kk, kr - 1), 0);
                rb[e] = q[TB ? cc * ld + kbc : kbc * ld + cc];
            } else {
                const int cc = min(c, ln - 1), kbc = min(kb, krem - 1);
                rb[e] = qb[TB ? cc * ldb + kbc : kbc * ldb + cc];
            }
        }
        krem_ld = krem;
        krem_ld2 = krem2;
        m_ld = lm;
        n_ld = ln;
    };
    auto store_stage = [&](int buf) {
        if (buf == 0)
            kst0 = krem_ld;
        else
            kst1 = krem_ld;
        kst0b = krem_ld2;
        // FP64 loads are already zero outside the block (guarded loads)
        constexpr bool guarded = std::is_same<T, double>::value;
        // valid depth and coefficient of the segment holding stage row k
        auto seg_krem = [&](int k) { return (KSV == 32 && k >= KP) ? krem_ld2 : krem_ld; };
        auto seg_k = [&](int k) { return KSV == 32 ? (k & (KP - 1)) : k; };
        auto a_val = [&](int e) {
            const int r = a_r + a_dr * e, ka = a_k + a_dk * e;
            const T al = (KSV == 32 && ka >= KP) ? alpha2 : alpha;
            const T fa = (guarded || (seg_k(ka) < seg_krem(ka) && r < m_ld)) ? al : (T)0;
            return fa * ra[e];
        };
        auto b_val = [&](int e) {
            const int c = b_c + b_dc * e, kb = b_k + b_dk * e;
            return (guarded || (seg_k(kb) < seg_krem(kb) && c < n_ld)) ? rb[e] : (T)0;
        };
        if constexpr (BF) {
#pragma unroll
            for (int e = 0; e < NEA; ++e) Ah[buf][a_r + a_dr * e][a_k + a_dk * e] = to_bf16(a_val(e));
#pragma unroll
            for (int e = 0; e < NEB; ++e) Bh[buf][b_c + b_dc * e][b_k + b_dk * e] = to_bf16(b_val(e));
        } else {
#pragma unroll
            for (int e = 0; e < NEA; ++e) {
                const int r = a_r + a_dr * e, ka = a_k + a_dk * e;
                const T al = (KSV == 32 && ka >= KP) ? alpha2 : alpha;
                const T fa = (guarded || (seg_k(ka) < seg_krem(ka) && r < m_ld)) ? al : (T)0;
                As[buf][ka][r] = fa * ra[e];
            }
#pragma unroll
            for (int e = 0; e < NEB; ++e) {
                const int c = b_c + b_dc * e, kb = b_k + b_dk * e;
                Bs[buf][kb][c] = (guarded || (seg_k(kb) < seg_krem(kb) && c < n_ld)) ? rb[e] : (T)0;
            }
        }
    };

    // Matrix-core work of one K stage.  ACT: the wave's 32 x 32 quadrant meets the
    // tile; R1 / C1: its second 16-row / 16-column block does.  Each combination is
    // its own straight-line code (chosen once per tile, wave-uniform), so the skipped
    // blocks cost nothing.  LDS operands of the next 4-deep step are read before the
    // MFMAs of the current one.
    auto mma_stage = [&](int buf, auto ACT, auto R1, auto C1) {
        if constexpr (ACT.value) {
            constexpr bool r1c = decltype(R1)::value, c1c = decltype(C1)::value;
            if constexpr (BF && KSV == 32) {
                // one v_mfma_f32_16x16x32_bf16 per 16 x 16 block and stage: lane l holds
                // 8 consecutive k of its row (A) and of its column (B), the same k for both
                const int kq = 8 * (lane >> 4), rl = lane & 15;
                const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(&Ah[buf][wr0 + rl][kq]);
                const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(&Bh[buf][wc0 + rl][kq]);
                bf16x8 a1 = {0, 0, 0, 0, 0, 0, 0, 0}, b1 = {0, 0, 0, 0, 0, 0, 0, 0};
                if constexpr (r1c) a1 = *reinterpret_cast<const bf16x8*>(&Ah[buf][wr0 + 16 + rl][kq]);
                if constexpr (c1c) b1 = *reinterpret_cast<const bf16x8*>(&Bh[buf][wc0 + 16 + rl][kq]);
                acc00 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc00, 0, 0, 0);
                if constexpr (c1c) acc01 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc01, 0, 0, 0);
                if constexpr (r1c) acc10 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc10, 0, 0, 0);
                if constexpr (r1c && c1c)
                    acc11 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc11, 0, 0, 0);
            } else if constexpr (BF) {
                const int kq = 4 * (lane >> 4), rl = lane & 15;
                const bf16x4 a0 = *reinterpret_cast<const bf16x4*>(&Ah[buf][wr0 + rl][kq]);
                const bf16x4 b0 = *reinterpret_cast<const bf16x4*>(&Bh[buf][wc0 + rl][kq]);
                bf16x4 a1 = {0, 0, 0, 0}, b1 = {0, 0, 0, 0};
                if constexpr (r1c) a1 = *reinterpret_cast<const bf16x4*>(&Ah[buf][wr0 + 16 + rl][kq]);
                if constexpr (c1c) b1 = *reinterpret_cast<const bf16x4*>(&Bh[buf][wc0 + 16 + rl][kq]);
                acc00 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b0, acc00, 0, 0, 0);
                if constexpr (c1c) acc01 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b1, acc01, 0, 0, 0);
                if constexpr (r1c) acc10 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b0, acc10, 0, 0, 0);
                if constexpr (r1c && c1c)
                    acc11 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b1, acc11, 0, 0, 0);
            } else {
                // 4-deep steps past the stage's valid depth (the zero padding of a
                // task's last stage) are skipped: a uniform branch per step.  KSV 32 runs
                // its two 16-deep segments one after the other, each with its own
                // operand registers, so no more of them are live than at KSV 16.
                constexpr int NH = KSV == 32 ? 2 : 1;   // segments of the stage
                constexpr int NK = (KSV == 32 ? 16 : KSV) / 4;  // 4-deep steps per segment
#pragma unroll
                for (int hs = 0; hs < NH; ++hs) {
                    // (two buffers: no skipping; a per-buffer depth would put the operand
                    // arrays in scratch)
                    const int kcur = NBUF == 1 ? (hs == 0 ? kst0 : kst0b) : KSV;
                    T a0[NK], a1[NK], b0[NK], b1[NK];
                    auto rd = [&](int ks) {
                        const int kr = hs * 16 + ks * 4 + (lane >> 4);
                        a0[ks] = As[buf][kr][wr0 + (lane & 15)];
                        b0[ks] = Bs[buf][kr][wc0 + (lane & 15)];
                        if constexpr (r1c) a1[ks] = As[buf][kr][wr0 + 16 + (lane & 15)];
                        if constexpr (c1c) b1[ks] = Bs[buf][kr][wc0 + 16 + (lane & 15)];
                    };
                    if (kcur <= 0) continue;  // (the stage's second segment may be empty)
                    rd(0);
#pragma unroll
                    for (int ks = 0; ks < NK; ++ks) {
                        if (ks * 4 >= kcur) continue;  // (no break: keeps the loop fully unrolled)
                        if (ks + 1 < NK && (ks + 1) * 4 < kcur) rd(ks + 1);
                        if constexpr (std::is_same<T, double>::value) {
                            acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[ks], b0[ks], acc00, 0, 0, 0);
                            if constexpr (c1c) acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[ks], b1[ks], acc01, 0, 0, 0);
                            if constexpr (r1c) acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[ks], b0[ks], acc10, 0, 0, 0);
                            if constexpr (r1c && c1c)
                                acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[ks], b1[ks], acc11, 0, 0, 0);
                        } else {
                            acc00 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[ks], b0[ks], acc00, 0, 0, 0);
                            if constexpr (c1c) acc01 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[ks], b1[ks], acc01, 0, 0, 0);
                            if constexpr (r1c) acc10 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[ks], b0[ks], acc10, 0, 0, 0);
                            if constexpr (r1c && c1c)
                                acc11 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[ks], b1[ks], acc11, 0, 0, 0);
                        }
                    }
                }
            }
        }
    };

    bind_loader(tl);
    if (tl.ktot > 0) load_stage();
    {
        const int m = tl.m, n = tl.n;
        const int nst = (tl.ktot + KSV - 1) / KSV;
        // 16 x 16 MFMA blocks wholly outside the tile's extent are skipped (wave-uniform
        // branches), so matrix-core work follows the block shape at 16 x 16 granularity
        const bool r1 = wr0 + 16 < m, c1 = wc0 + 16 < n;
        const bool any = wr0 < m && wc0 < n;
        acc00 = acc_t{0, 0, 0, 0};
        acc01 = acc_t{0, 0, 0, 0};
        acc10 = acc_t{0, 0, 0, 0};
        acc11 = acc_t{0, 0, 0, 0};
        auto run = [&](auto ACT, auto R1, auto C1) {
            if (nst <= 0) return;
            store_stage(0);
            __syncthreads();
            for (int s = 0; s < nst; ++s) {
                const int buf = NBUF == 2 ? (s & 1) : 0;
                if (s + 1 < nst) load_stage();
                mma_stage(buf, ACT, R1, C1);
                if constexpr (NBUF == 2) {
                    if (s + 1 < nst) store_stage(buf ^ 1);
                    __syncthreads();
                } else {
                    __syncthreads();
                    if (s + 1 < nst) {
                        store_stage(0);
                        __syncthreads();
                    }
                }
            }
        };
        using F = std::false_type;
        using Tr = std::true_type;
        if (!any)
            run(F{}, F{}, F{});
        else if (r1 && c1)
            run(Tr{}, Tr{}, Tr{});
        else if (r1)
            run(Tr{}, Tr{}, F{});
        else if (c1)
            run(Tr{}, F{}, Tr{});
        else
            run(Tr{}, F{}, F{});

        // epilogue (lane layouts measured on gfx950): v_mfma_f64_16x16x4_f64 gives lane l
        // rows l/16 + 4v of column l%16; v_mfma_f32_16x16x4_f32 and
        // v_mfma_f32_16x16x16_bf16 rows 4(l/16) + v.
        T* C = space_ptr<T, NSP>(B, tl.flags & 0xff) + tl.coff;
        const int ldc = tl.ldc;
        const bool beta = ((tl.flags >> 8) & 0xff) != 0;
        auto put = [&](const acc_t& a, int rb0_, int cb0) {
            const int col = cb0 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = std::is_same<T, double>::value ? rb0_ + (lane >> 4) + 4 * v : rb0_ + 4 * (lane >> 4) + v;
                if (row < m && col < n) {
                    T* p = C + (int64_t)row * ldc + col;
                    *p = beta ? (*p + a[v]) : a[v];
                }
            }
        };
        put(acc00, wr0, wc0);
        put(acc01, wr0, wc0 + 16);
        put(acc10, wr0 + 16, wc0);
        put(acc11, wr0 + 16, wc0 + 16);
    }
}

// Single-wave variant for blocks of at most 32 x 32 (SH_SMALL tiles): one wavefront
// computes a 32 x 32 tile (2 x 2 MFMA blocks) over its task list with 16-deep K stages
// staged through one LDS buffer, the same arithmetic and summation order as bsgemm's
// quadrant.  FP64 or FP32 operands (no BF16 rounding).
template <typename T, bool TA, bool TB, int NSP>
__global__ __launch_bounds__(64) void bsgemm_w1(const Tile* __restrict__ tiles, const Task* __restrict__ tasks,
                                                BasesT<T> B) {
    using acc_t = typename std::conditional<std::is_same<T, double>::value, dbl4, flt4>::type;
    constexpr int KSV = 16, TS = 32, NE = TS * KSV / 64;  // 8 elements of A and of B per lane
    __shared__ T As[KSV][TS + LDS_PAD];
    __shared__ T Bs[KSV][TS + LDS_PAD];
    const int lane = threadIdx.x;
    // load lanes (element e: idx = lane + 64 e): A !TA: k = idx % 16, row = idx / 16;
    // A TA: row = idx % 32, k = idx / 32; B !TB: col = idx % 32, k = idx / 32;
    // B TB: k = idx % 16, col = idx / 16
    const int a_r = TA ? (lane % TS) : (lane / KSV);
    const int a_k = TA ? (lane / TS) : (lane % KSV);
    const int b_c = TB ? (lane / KSV) : (lane % TS);
    const int b_k = TB ? (lane % KSV) : (lane / TS);
    constexpr int a_dr = TA ? 0 : 64 / KSV, a_dk = TA ? 64 / TS : 0;
    constexpr int b_dc = TB ? 64 / KSV : 0, b_dk = TB ? 0 : 64 / TS;

    const Tile tl = tiles[blockIdx.x];
    const int m = tl.m, n = tl.n;
    Cursor<T, TA, TB, NSP, KSV> cur;
    cur.start(tl.tbeg, tl.tend, tasks, B, tl.r0, tl.c0);
    T ra[NE], rb[NE];
    T alpha = 0;
    int krem_ld = 0;
    auto load_stage = [&]() {
        const T *qa, *qb;
        int krem;
        cur.next(tasks, B, tl.r0, tl.c0, qa, qb, krem, alpha);
        const int lda = cur.lda, ldb = cur.ldb;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int r = a_r + a_dr * e, ka = a_k + a_dk * e;
            T va = 0;
            if (ka < krem && r < m) va = qa[TA ? ka * lda + r : r * lda + ka];
            ra[e] = va;
        }
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int c = b_c + b_dc * e, kb = b_k + b_dk * e;
            T vb = 0;
            if (kb < krem && c < n) vb = qb[TB ? c * ldb + kb : kb * ldb + c];
            rb[e] = vb;
        }
        krem_ld = krem;
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int e = 0; e < NE; ++e) As[a_k + a_dk * e][a_r + a_dr * e] = alpha * ra[e];
#pragma unroll
        for (int e = 0; e < NE; ++e) Bs[b_k + b_dk * e][b_c + b_dc * e] = rb[e];
    };
    acc_t acc00 = {0, 0, 0, 0}, acc01 = {0, 0, 0, 0}, acc10 = {0, 0, 0, 0}, acc11 = {0, 0, 0, 0};
    const bool r1 = 16 < m, c1 = 16 < n;
    const int nst = tl.ktot / KSV;
    if (nst > 0) load_stage();
    for (int s = 0; s < nst; ++s) {
        store_stage();
        const int kcur = krem_ld;
        __syncthreads();
        if (s + 1 < nst) load_stage();
#pragma unroll
        for (int ks = 0; ks < KSV / 4; ++ks) {
            if (ks * 4 >= kcur) continue;
            const int kr = ks * 4 + (lane >> 4);
            const T a0 = As[kr][lane & 15], b0 = Bs[kr][lane & 15];
            const T a1 = r1 ? As[kr][16 + (lane & 15)] : (T)0;
            const T b1 = c1 ? Bs[kr][16 + (lane & 15)] : (T)0;
            if constexpr (std::is_same<T, double>::value) {
                acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc00, 0, 0, 0);
                if (c1) acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc01, 0, 0, 0);
                if (r1) acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc10, 0, 0, 0);
                if (r1 && c1) acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc11, 0, 0, 0);
            } else {
                acc00 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc00, 0, 0, 0);
                if (c1) acc01 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc01, 0, 0, 0);
                if (r1) acc10 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc10, 0, 0, 0);
                if (r1 && c1) acc11 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc11, 0, 0, 0);
            }
        }
        __syncthreads();
    }
    T* C = space_ptr<T, NSP>(B, tl.flags & 0xff) + tl.coff;
    const int ldc = tl.ldc;
    const bool beta = ((tl.flags >> 8) & 0xff) != 0;
    auto put = [&](const acc_t& a, int rb0_, int cb0) {
        const int col = cb0 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = std::is_same<T, double>::value ? rb0_ + (lane >> 4) + 4 * v : rb0_ + 4 * (lane >> 4) + v;
            if (row < m && col < n) {
                T* p = C + (int64_t)row * ldc + col;
                *p = beta ? (*p + a[v]) : a[v];
            }
        }
    };
    put(acc00, 0, 0);
    put(acc01, 0, 16);
    put(acc10, 16, 0);
    put(acc11, 16, 16);
}

// Fixed-order sum of split-K partial tiles into the owning output tile.  Block
// (x, y) sums the y-th of gridDim.y slices of tile x's elements; the partials of an
// element are added in index order (loads issued four at a time).
template <typename T>
__global__ __launch_bounds__(256) void reduce_partials(const Reduce* __restrict__ red, BasesT<T> B) {
    const Reduce r = red[blockIdx.x];
    const T* P = B.p[SP_PART] + r.pbase;
    T* C = space_ptr(B, r.cspace) + r.coff;
    const int total = r.m * r.n;
    const int slice = (total + (int)gridDim.y - 1) / (int)gridDim.y;
    const int e1 = min(total, slice * ((int)blockIdx.y + 1));
    for (int e = slice * (int)blockIdx.y + (int)threadIdx.x; e < e1; e += blockDim.x) {
        const int row = e / r.n, col = e % r.n;
        const T* q = P + row * r.pld + col;
        T acc = 0;
        int j = 0;
        for (; j + 4 <= r.np; j += 4) {
            const T p0 = q[(int64_t)j * TM * TN], p1 = q[(int64_t)(j + 1) * TM * TN];
            const T p2 = q[(int64_t)(j + 2) * TM * TN], p3 = q[(int64_t)(j + 3) * TM * TN];
            acc += p0;
            acc += p1;
            acc += p2;
            acc += p3;
        }
        for (; j < r.np; ++j) acc += q[(int64_t)j * TM * TN];
        T* p = C + (int64_t)row * r.ldc + col;
        *p = r.beta ? (*p + acc) : acc;
    }
}

// dst[j] = src[idx[j]] / dst[idx[j]] = src[j] for j < n; indices outside [0, nsrc) /
// [0, ndst) are skipped (the element is left unchanged).
__global__ void gather_index(int64_t n, const int64_t* __restrict__ idx, int64_t nsrc, const double* __restrict__ src,
                             double* __restrict__ dst) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx[e];
        if (i >= 0 && i < nsrc) dst[e] = src[i];
    }
}

__global__ void scatter_index(int64_t n, const int64_t* __restrict__ idx, int64_t ndst, const double* __restrict__ src,
                              double* __restrict__ dst) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx[e];
        if (i >= 0 && i < ndst) dst[i] = src[e];
    }
}

// y += a x
__global__ void axpy_f64(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] += a * x[e];
}

__global__ void cvt_f64_f32(int64_t n, const double* __restrict__ s, float* __restrict__ d) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = (float)s[i];
}

__global__ void cvt_f32_f64(int64_t n, const float* __restrict__ s, double* __restrict__ d) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        d[i] = (double)s[i];
}

template <typename T>
__global__ void gather_scale(const Gather* __restrict__ g, BasesT<T> B) {
    const Gather gg = g[blockIdx.x];
    const T* s = space_ptr(B, gg.sspace) + gg.soff;
    T* d = space_ptr(B, gg.dspace) + gg.doff;
    for (int x = threadIdx.x; x < gg.count; x += blockDim.x)
        d[(int64_t)x * gg.dstride] = (T)gg.alpha * s[(int64_t)x * gg.sstride];
}

// Whole-payload copies (Gather entries with long counts): blockIdx.x picks the entry,
// the gridDim.y blocks of 256 threads split its elements.
template <typename T>
__global__ void copy_wide(const Gather* __restrict__ g, BasesT<T> B) {
    const Gather gg = g[blockIdx.x];
    const T* s = space_ptr(B, gg.sspace) + gg.soff;
    T* d = space_ptr(B, gg.dspace) + gg.doff;
    for (int64_t x = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; x < gg.count;
         x += (int64_t)gridDim.y * blockDim.x)
        d[x * gg.dstride] = (T)gg.alpha * s[x * gg.sstride];
}

template <typename T>
__global__ void fill_zero(T* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (T)0;
}

// ---------------------------------------------------------------- Davidson

constexpr int DOT_BLOCKS = 256;
constexpr int DOT_THREADS = 256;
constexpr int KMAX = 32;

// Deterministic dots: pass 1 writes per-block partial sums, pass 2 sums them in
// a fixed tree order.  part[blk * KMAX + j].
// Sum of v over the 64 lanes of a wavefront (butterfly: every lane holds the sum,
// in an order fixed by the lane pattern).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// part[block][j] = partial a_j . b over the block's grid-stride elements, j < k:
// one sweep over b (each a_j and b read once), k sums per thread in registers, then
// per j a wavefront sum and a fixed-order sum over the block's 4 wavefronts.
__global__ __launch_bounds__(DOT_THREADS) void dots_pass1(int64_t n, int k, const double* __restrict__ a,
                                                          int64_t lda, const double* __restrict__ b,
                                                          double* __restrict__ part) {
    __shared__ double red[DOT_THREADS / 64][KMAX];
    double s[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) s[j] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * DOT_THREADS + threadIdx.x; e < n; e += (int64_t)DOT_BLOCKS * DOT_THREADS) {
        const double bv = b[e];
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < k) s[j] += a[(int64_t)j * lda + e] * bv;
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        if (j < k) {
            const double t = wave_sum(s[j]);
            if (lane == 0) red[w][j] = t;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < k) {
        double t = red[0][threadIdx.x];
        for (int q = 1; q < DOT_THREADS / 64; ++q) t += red[q][threadIdx.x];
        part[blockIdx.x * KMAX + threadIdx.x] = t;
    }
}

// out[j * ostride] = sum over the DOT_BLOCKS partials of dot j (fixed order).
__global__ __launch_bounds__(DOT_BLOCKS) void dots_pass2(int k, const double* __restrict__ part, double* out,
                                                         int ostride) {
    __shared__ double red[DOT_BLOCKS / 64][KMAX];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int j = 0; j < k; ++j) {
        const double t = wave_sum(part[threadIdx.x * KMAX + j]);
        if (lane == 0) red[w][j] = t;
    }
    __syncthreads();
    if ((int)threadIdx.x < k) {
        double t = red[0][threadIdx.x];
        for (int q = 1; q < DOT_BLOCKS / 64; ++q) t += red[q][threadIdx.x];
        out[(int64_t)threadIdx.x * ostride] = t;
    }
}

// Davidson workspace (doubles):
//   [0, 1024)         G (KMAX x KMAX, row-major; G[i][j] = v_i . s_j)
//   [1024, 1056)      y
//   [1056, 1088)      c (Gram-Schmidt coefficients)
//   [1088, 1096)      scalars: theta, |r|^2, |t|^2, ...
//   [1096, ...)       partial sums (DOT_BLOCKS x KMAX)
//   then              Q (KMAX x KMAX): eigenvectors of the last eigensolve, columns
//                     (Q[i][j] = component i of eigenvector j); then k of that solve
constexpr int64_t DW_G = 0, DW_Y = 1024, DW_C = 1056, DW_S = 1088, DW_P = 1096;
constexpr int64_t DW_Q = DW_P + (int64_t)DOT_BLOCKS * KMAX, DW_KQ = DW_Q + (int64_t)KMAX * KMAX;
constexpr int64_t DW_TOTAL = DW_KQ + 1;

// Lowest eigenpair of the symmetrised k x k projected matrix by Jacobi rotations
// (one wavefront).  Each step rotates k/2 disjoint index pairs at once (round-robin
// pairing, k - 1 steps per sweep, a dummy index when k is odd): one lane computes each
// pair's rotation, then the row and the column updates of all pairs run in parallel.
// The rotations start from an orthogonal basis W and act on W^T A W, so the
// accumulated W R holds the eigenvectors of A for any orthogonal W.  When the last
// solve was for k - 1 (the basis grew by one vector, the leading block of A is
// unchanged) W = diag(Q, 1) with that solve's eigenvectors Q: W^T A W is then diagonal
// but for its last row and column, and few sweeps remain.  Q is used only if its
// columns are orthonormal to 1e-12; otherwise W = I.
// theta -> ws[DW_S], y -> ws[DW_Y..]; all eigenvectors -> ws[DW_Q..], k -> ws[DW_KQ].
__global__ __launch_bounds__(64) void dav_eig(int k, double* ws, double* scal) {
    __shared__ double A[KMAX][KMAX + 1];
    __shared__ double V[KMAX][KMAX + 1];
    __shared__ double C[KMAX][KMAX + 1];
    __shared__ double rc[KMAX / 2], rs[KMAX / 2];
    __shared__ int rp[KMAX / 2], rq[KMAX / 2];
    const int t = threadIdx.x;
    const int ke = (k + 1) & ~1;
    const int np = ke / 2;
    // round-robin pairing: index 0 stays, indices 1 .. ke-1 rotate by one place per
    // step (the identity again after ke - 1 steps, i.e. at every sweep), so the
    // index at position i in step `step` has a closed form
    auto order = [ke](int i, int step) {
        const int m = ke - 1;
        return i == 0 ? 0 : 1 + ((i - 1 - step) % m + m) % m;
    };
    const double* G = ws + DW_G;
    double* Q = ws + DW_Q;
    const int kw = (k >= 2 && ws[DW_KQ] == (double)(k - 1)) ? k - 1 : 0;  // warm-start block
    for (int idx = t; idx < k * k; idx += 64) {
        int i = idx / k, j = idx % k;
        A[i][j] = 0.5 * (G[i * KMAX + j] + G[j * KMAX + i]);
        V[i][j] = (i < kw && j < kw) ? Q[i * KMAX + j] : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    if (kw > 0) {
        // W = diag(Q, 1) must be orthogonal: max |W^T W - I|
        double dev = 0.0;
        for (int idx = t; idx < k * k; idx += 64) {
            const int i = idx / k, j = idx % k;
            double g = 0.0;
            for (int l = 0; l < k; ++l) g += V[l][i] * V[l][j];
            dev = fmax(dev, fabs(g - (i == j ? 1.0 : 0.0)));
        }
        for (int m = 32; m > 0; m >>= 1) dev = fmax(dev, __shfl_xor(dev, m));
        if (dev <= 1e-12) {  // (the same on every lane)
            for (int idx = t; idx < k * k; idx += 64) {  // C = A W
                const int i = idx / k, j = idx % k;
                double g = 0.0;
                for (int l = 0; l < k; ++l) g += A[i][l] * V[l][j];
                C[i][j] = g;
            }
            __syncthreads();
            for (int idx = t; idx < k * k; idx += 64) {  // A = W^T C (A is free now)
                const int i = idx / k, j = idx % k;
                double g = 0.0;
                for (int l = 0; l < k; ++l) g += V[l][i] * C[l][j];
                A[i][j] = g;
            }
            __syncthreads();
            for (int idx = t; idx < k * k; idx += 64) {  // symmetrised copy ...
                const int i = idx / k, j = idx % k;
                C[i][j] = 0.5 * (A[i][j] + A[j][i]);
            }
            __syncthreads();
            for (int idx = t; idx < k * k; idx += 64) A[idx / k][idx % k] = C[idx / k][idx % k];  // ... back
        } else {
            for (int idx = t; idx < k * k; idx += 64) {
                const int i = idx / k, j = idx % k;
                V[i][j] = (i == j) ? 1.0 : 0.0;
            }
        }
        __syncthreads();
    }
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int idx = t; idx < k * k; idx += 64) {
            const int i = idx / k, j = idx % k;
            const double v = fabs(A[i][j]);
            if (i == j)
                dia = fmax(dia, v);
            else
                off = fmax(off, v);
        }
        for (int m = 32; m > 0; m >>= 1) {
            off = fmax(off, __shfl_xor(off, m));
            dia = fmax(dia, __shfl_xor(dia, m));
        }
        if (off <= 1e-16 * fmax(dia, 1e-300)) break;  // the same on every lane
        for (int step = 0; step < ke - 1; ++step) {
            if (t < np) {
                int p = order(t, step), q = order(ke - 1 - t, step);
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
                double c = 1.0, sn = 0.0;
                if (q < k) {
                    const double apq = A[p][q];
                    if (fabs(apq) >= 1e-300) {
                        const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
                        const double tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(tt * tt + 1.0);
                        sn = tt * c;
                    }
                }
                rp[t] = p;
                rq[t] = q;
                rc[t] = c;
                rs[t] = sn;
            }
            __syncthreads();
            for (int idx = t; idx < np * k; idx += 64) {  // rows p, q of every pair
                const int pi = idx / k, j = idx % k;
                const int p = rp[pi], q = rq[pi];
                if (q >= k || rs[pi] == 0.0) continue;
                const double c = rc[pi], sn = rs[pi];
                const double ap = A[p][j], aq = A[q][j];
                A[p][j] = c * ap - sn * aq;
                A[q][j] = sn * ap + c * aq;
            }
            __syncthreads();
            for (int idx = t; idx < np * k; idx += 64) {  // columns p, q of A and V
                const int pi = idx / k, i = idx % k;
                const int p = rp[pi], q = rq[pi];
                if (q >= k || rs[pi] == 0.0) continue;
                const double c = rc[pi], sn = rs[pi];
                const double ap = A[i][p], aq = A[i][q];
                A[i][p] = c * ap - sn * aq;
                A[i][q] = sn * ap + c * aq;
                const double vp = V[i][p], vq = V[i][q];
                V[i][p] = c * vp - sn * vq;
                V[i][q] = sn * vp + c * vq;
            }
            __syncthreads();
            if (t < np && rq[t] < k && rs[t] != 0.0) {  // the rotated pair's element is zero
                A[rp[t]][rq[t]] = 0.0;
                A[rq[t]][rp[t]] = 0.0;
            }
            __syncthreads();
        }
    }
    for (int idx = t; idx < k * k; idx += 64) Q[(idx / k) * KMAX + idx % k] = V[idx / k][idx % k];
    if (t == 0) {
        ws[DW_KQ] = (double)k;
        int best = 0;
        for (int i = 1; i < k; ++i)
            if (A[i][i] < A[best][best]) best = i;
        int big = 0;
        for (int i = 1; i < k; ++i)
            if (fabs(V[i][best]) > fabs(V[big][best])) big = i;
        double sg = V[big][best] < 0 ? -1.0 : 1.0;
        double nrm = 0.0;
        for (int i = 0; i < k; ++i) nrm += V[i][best] * V[i][best];
        nrm = sqrt(nrm);
        for (int i = 0; i < k; ++i) ws[DW_Y + i] = sg * V[i][best] / nrm;
        ws[DW_S + 0] = A[best][best];
        scal[0] = A[best][best];
    }
}

// x = V^T y, hx = S^T y, t = hx - theta x
__global__ void dav_combine(int64_t n, int k, const double* __restrict__ V, int64_t ldv, const double* __restrict__ S,
                            int64_t lds, const double* __restrict__ ws, double* __restrict__ x, double* __restrict__ hx,
                            double* __restrict__ t) {
    __shared__ double y[KMAX];
    __shared__ double theta;
    if (threadIdx.x < k) y[threadIdx.x] = ws[DW_Y + threadIdx.x];
    if (threadIdx.x == 0) theta = ws[DW_S + 0];
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double xv = 0.0, hv = 0.0;
        for (int j = 0; j < k; ++j) {
            xv += y[j] * V[(int64_t)j * ldv + e];
            hv += y[j] * S[(int64_t)j * lds + e];
        }
        x[e] = xv;
        hx[e] = hv;
        t[e] = hv - theta * xv;
    }
}

// t = t / guard(theta - diag)
__global__ void dav_precond(int64_t n, const double* __restrict__ diag, double guard, const double* __restrict__ ws,
                            double* __restrict__ t) {
    const double theta = ws[DW_S + 0];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double den = theta - diag[e];
        if (fabs(den) < guard) den = den < 0 ? -guard : guard;
        t[e] = t[e] / den;
    }
}

// t -= sum_j c_j v_j
__global__ void dav_project(int64_t n, int k, const double* __restrict__ V, int64_t ldv, const double* __restrict__ ws,
                            double* __restrict__ t) {
    __shared__ double c[KMAX];
    if (threadIdx.x < k) c[threadIdx.x] = ws[DW_C + threadIdx.x];
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double acc = t[e];
        for (int j = 0; j < k; ++j) acc -= c[j] * V[(int64_t)j * ldv + e];
        t[e] = acc;
    }
}

// v -= c x and s -= c hx with c = *cp (one Gram-Schmidt pass against the Ritz vector)
__global__ void restart_combine(int64_t n, const double* __restrict__ x, const double* __restrict__ hx, double* v,
                                double* sv, const double* cp) {
    const double c = *cp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        v[e] -= c * x[e];
        sv[e] -= c * hx[e];
    }
}

// v, sv /= sqrt(*nu2) when the norm is not negligible, else both zero; scal[3] = norm
__global__ void restart_scale(int64_t n, double* v, double* sv, const double* nu2, double* scal) {
    const double nu = sqrt(fmax(*nu2, 0.0));
    const double inv = nu > 1e-10 ? 1.0 / nu : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        v[e] *= inv;
        sv[e] *= inv;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[3] = nu > 1e-10 ? nu : 0.0;
}

// t /= sqrt(ws[DW_S+2]) (if > 0); scal[1] = sqrt(|r|^2), scal[2] = |t|
__global__ void dav_finish(int64_t n, double* ws, double* __restrict__ t, double* scal) {
    const double tn = sqrt(ws[DW_S + 2]);
    const double inv = tn > 0 ? 1.0 / tn : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        t[e] *= inv;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[1] = sqrt(ws[DW_S + 1]);
        scal[2] = tn;
    }
}

// ---------------------------------------------------------------- host side

static int hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return HX_EHIP;
    }
    return HX_OK;
}

static Bases make_bases(const Plan* P, const double* psi, double* out, const double* L, const double* R, void* ws) {
    Bases b{};
    b.p[SP_PSI] = const_cast<double*>(psi);
    b.p[SP_OUT] = out;
    b.p[SP_L] = const_cast<double*>(L);
    b.p[SP_R] = const_cast<double*>(R);
    b.p[SP_WS] = static_cast<double*>(ws);
    b.p[SP_TAB] = reinterpret_cast<double*>(static_cast<char*>(P->dev) + P->off_coef);
    b.p[SP_PART] = ws ? static_cast<double*>(ws) + P->part_base : nullptr;
    return b;
}

template <typename T, int NSP, int KSV, int NBUF, bool BF = false, int WR = 2>
static int launch_kind(int kind, int64_t ntile, const Tile* tiles, const Task* tasks, const BasesT<T>& B,
                       hipStream_t s) {
    const dim3 block(256);
    const dim3 grid((unsigned)ntile);
    const int nt = (int)ntile;
    switch (kind) {
        case NN:
            hipLaunchKernelGGL((bsgemm<T, false, false, NSP, KSV, NBUF, BF, WR>), grid, block, 0, s, tiles,
                               tasks, B, nt);
            return HX_OK;
        case NT:
            hipLaunchKernelGGL((bsgemm<T, false, true, NSP, KSV, NBUF, BF, WR>), grid, block, 0, s, tiles,
                               tasks, B, nt);
            return HX_OK;
        case TN_:
            hipLaunchKernelGGL((bsgemm<T, true, false, NSP, KSV, NBUF, BF, WR>), grid, block, 0, s, tiles,
                               tasks, B, nt);
            return HX_OK;
        default:
            set_error("internal: bad GEMM kind");
            return HX_EINVAL;
    }
}

// Launch check, then the split-K reduction of the launch (if any).
template <typename T>
static int finish_gemm(const Plan* P, const Launch& L, const BasesT<T>& B, hipStream_t s) {
    int rc = hip_check(hipGetLastError(), "bsgemm launch");
    if (rc || L.nred <= 0) return rc;
    const Reduce* red = reinterpret_cast<const Reduce*>(static_cast<const char*>(P->dev) + P->off_reduces) + L.red0;
    hipLaunchKernelGGL((reduce_partials<T>), dim3((unsigned)L.nred, 8), dim3(256), 0, s, red, B);
    return hip_check(hipGetLastError(), "reduce launch");
}

template <typename T, int NSP = NSP_FWD, bool BF = false>
static int launch_gemm(const Plan* P, const Launch& L, const BasesT<T>& B, hipStream_t s) {
    if (L.ntile <= 0) return HX_OK;
    const Tile* tiles = reinterpret_cast<const Tile*>(static_cast<const char*>(P->dev) + P->off_tiles) + L.tile0;
    const Task* tasks = reinterpret_cast<const Task*>(static_cast<const char*>(P->dev) + P->off_tasks);
    if (L.ntile > INT32_MAX) {
        set_error("launch has more than 2^31 tiles");
        return HX_EINVAL;
    }
    const int64_t nt = L.ntile;
    int rk;
    if (L.shape != SH_SQ && !((L.shape == SH_SMALL) ? P->variant == 6 : (P->variant == 4 || P->variant == 5))) {
        set_error("internal: tile shape without its kernel variant");
        return HX_EINVAL;
    }
    // the wave layout of the launch's tile shape (64 x 64 unless variant 4 or 5)
    auto shaped = [&](auto KIND_NBUF, auto BFC) -> int {
        constexpr int NB = decltype(KIND_NBUF)::value;
        constexpr bool BFv = decltype(BFC)::value;
        // BF16 products with one LDS buffer: 32-deep stages (two 16-deep segments of
        // the plan) on the full-rate v_mfma_f32_16x16x32_bf16.  (FP32 products in
        // 32-deep stages measured slower: 86-94 registers, 5 waves per SIMD against 8.)
        constexpr int KS = (BFv && NB == 1) ? 32 : 16;
        switch (L.shape) {
            case SH_TALL:
                return launch_kind<T, NSP, KS, NB, BFv, 4>(L.kind, nt, tiles, tasks, B, s);
            case SH_WIDE:
                return launch_kind<T, NSP, KS, NB, BFv, 1>(L.kind, nt, tiles, tasks, B, s);
            default:
                return launch_kind<T, NSP, KS, NB, BFv, 2>(L.kind, nt, tiles, tasks, B, s);
        }
    };
    using One = std::integral_constant<int, 1>;
    using Two = std::integral_constant<int, 2>;
    using BFc = std::integral_constant<bool, BF>;
    if constexpr (BF) {
        switch (P->variant) {
            case 1:
            case 5:
                rk = shaped(One{}, BFc{});
                break;
            case 6:
                if (L.shape == SH_SMALL) {
                    set_error("BF16 products have no single-wave tiles (kernel variant 6)");
                    return HX_EUNSUP;
                }
                rk = shaped(One{}, BFc{});
                break;
            case 0:
            case 4:
                rk = shaped(Two{}, BFc{});
                break;
            default:
                set_error("BF16 products need a 16-deep kernel variant (not 2)");
                return HX_EUNSUP;
        }
        if (rk) return rk;
        return finish_gemm(P, L, B, s);
    }
    switch (P->variant) {
        case 1:
        case 5:
            rk = shaped(One{}, BFc{});
            break;
        case 2:
            rk = launch_kind<T, NSP, 8, 2>(L.kind, nt, tiles, tasks, B, s);
            break;
        case 6:
            if (L.shape == SH_SMALL) {
                const dim3 grid((unsigned)nt), block(64);
                switch (L.kind) {
                    case NN:
                        hipLaunchKernelGGL((bsgemm_w1<T, false, false, NSP>), grid, block, 0, s, tiles, tasks, B);
                        break;
                    case NT:
                        hipLaunchKernelGGL((bsgemm_w1<T, false, true, NSP>), grid, block, 0, s, tiles, tasks, B);
                        break;
                    case TN_:
                        hipLaunchKernelGGL((bsgemm_w1<T, true, false, NSP>), grid, block, 0, s, tiles, tasks, B);
                        break;
                    default:
                        set_error("internal: bad GEMM kind");
                        return HX_EINVAL;
                }
                rk = HX_OK;
            } else {
                rk = shaped(One{}, BFc{});
            }
            break;
        default:
            rk = shaped(Two{}, BFc{});
            break;
    }
    if (rk) return rk;
    return finish_gemm(P, L, B, s);
}

static inline hipStream_t s_of(hx_stream st) { return static_cast<hipStream_t>(st); }

static int check_ready(const hx_plan* plan, int kind, int kind2 = -1) {
    if (!plan) {
        set_error("null plan");
        return HX_EINVAL;
    }
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if (!P->dev) {
        set_error("plan not uploaded (call hx_plan_upload first)");
        return HX_EINVAL;
    }
    if (kind >= 0 && P->kind != kind && P->kind != kind2 && !(kind == PK_ENV_LEFT && P->kind == PK_ENV_RIGHT)) {
        set_error("plan kind does not match this entry point");
        return HX_EINVAL;
    }
    return HX_OK;
}

extern "C" {

int hx_plan_upload(hx_plan* plan, void* dev_tables, hx_stream stream) {
    if (!plan || !dev_tables) {
        set_error("plan_upload: null argument");
        return HX_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(dev_tables) & 255) != 0) {
        set_error("plan_upload: table buffer must be 256-byte aligned");
        return HX_EINVAL;
    }
    Plan* P = reinterpret_cast<Plan*>(plan);
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* d = static_cast<char*>(dev_tables);
    int rc;
    if (!P->tiles.empty() &&
        (rc = hip_check(hipMemcpyAsync(d + P->off_tiles, P->tiles.data(), P->tiles.size() * sizeof(Tile),
                                       hipMemcpyHostToDevice, s), "upload tiles")))
        return rc;
    if (!P->tasks.empty() &&
        (rc = hip_check(hipMemcpyAsync(d + P->off_tasks, P->tasks.data(), P->tasks.size() * sizeof(Task),
                                       hipMemcpyHostToDevice, s), "upload tasks")))
        return rc;
    if (!P->gathers.empty() &&
        (rc = hip_check(hipMemcpyAsync(d + P->off_gathers, P->gathers.data(), P->gathers.size() * sizeof(Gather),
                                       hipMemcpyHostToDevice, s), "upload gathers")))
        return rc;
    if (!P->coef.empty() &&
        (rc = hip_check(hipMemcpyAsync(d + P->off_coef, P->coef.data(), P->coef.size() * sizeof(double),
                                       hipMemcpyHostToDevice, s), "upload coefficients")))
        return rc;
    if (!P->reduces.empty() &&
        (rc = hip_check(hipMemcpyAsync(d + P->off_reduces, P->reduces.data(), P->reduces.size() * sizeof(Reduce),
                                       hipMemcpyHostToDevice, s), "upload reductions")))
        return rc;
    if ((rc = hip_check(hipStreamSynchronize(s), "upload sync"))) return rc;
    P->dev = dev_tables;
    return HX_OK;
}

// The mixing GEMMs, then the copies that stack the first-round operands of merged
// intermediates (read from the mixed operators and the right environment).
static int run_prepare(const Plan* P, const Bases& B, hipStream_t s) {
    int rc;
    for (const Launch& l : P->prep)
        if ((rc = launch_gemm(P, l, B, s))) return rc;
    const Gather* g = reinterpret_cast<const Gather*>(static_cast<const char*>(P->dev) + P->off_gathers);
    for (const GatherLaunch& gl : P->prep_gather) {
        hipLaunchKernelGGL(gather_scale<double>, dim3((unsigned)gl.ng), dim3(256), 0, s, g + gl.g0, B);
        if ((rc = hip_check(hipGetLastError(), "stacked operand copies"))) return rc;
    }
    return HX_OK;
}

int hx_heff_prepare(const hx_plan* plan, const double* L, const double* R, void* ws, hx_stream stream) {
    int rc = check_ready(plan, PK_HEFF, PK_HEFF_VJP);
    if (rc) return rc;
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if ((P->in_nnz && !L) || (P->in2_nnz && !R) || (P->ws_doubles && !ws)) {
        set_error("heff_prepare: null operand");
        return HX_EINVAL;
    }
    Bases B = make_bases(P, nullptr, nullptr, L, R, ws);
    return run_prepare(P, B, static_cast<hipStream_t>(stream));
}

int hx_heff_apply(const hx_plan* plan, const double* L, const double* R, void* ws, const double* psi, double* sigma,
                  hx_stream stream) {
    int rc = check_ready(plan, PK_HEFF);
    if (rc) return rc;
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if ((P->psi_nnz && (!psi || !sigma)) || (P->in_nnz && !L) || (P->in2_nnz && !R) || (P->ws_doubles && !ws)) {
        set_error("heff_apply: null operand");
        return HX_EINVAL;
    }
    if (P->psi_nnz && psi == sigma) {
        set_error("heff_apply: psi and sigma must not alias");
        return HX_EINVAL;
    }
    Bases B = make_bases(P, psi, sigma, L, R, ws);
    for (const Launch& l : P->apply)
        if ((rc = launch_gemm(P, l, B, static_cast<hipStream_t>(stream)))) return rc;
    return HX_OK;
}

static int cvt(int64_t n, const double* a, float* b, hipStream_t s) {
    if (n <= 0) return HX_OK;
    const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(cvt_f64_f32, dim3(nb), dim3(256), 0, s, n, a, b);
    return hip_check(hipGetLastError(), "convert f64->f32");
}

int hx_convert_f64_f32(int64_t n, const double* src, float* dst, hx_stream stream) {
    if (n < 0 || (n > 0 && (!src || !dst))) {
        set_error("convert: bad arguments");
        return HX_EINVAL;
    }
    return cvt(n, src, dst, static_cast<hipStream_t>(stream));
}

int hx_convert_f32_f64(int64_t n, const float* src, double* dst, hx_stream stream) {
    if (n < 0 || (n > 0 && (!src || !dst))) {
        set_error("convert: bad arguments");
        return HX_EINVAL;
    }
    if (n == 0) return HX_OK;
    const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(cvt_f32_f64, dim3(nb), dim3(256), 0, static_cast<hipStream_t>(stream), n, src, dst);
    return hip_check(hipGetLastError(), "convert f32->f64");
}

int hx_gather_index(int64_t n, const int64_t* idx, int64_t nsrc, const double* src, double* dst, hx_stream stream) {
    if (n < 0 || nsrc < 0 || (n > 0 && (!idx || !dst || (nsrc > 0 && !src)))) {
        set_error("gather_index: bad arguments");
        return HX_EINVAL;
    }
    if (n == 0) return HX_OK;
    const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(gather_index, dim3(nb), dim3(256), 0, static_cast<hipStream_t>(stream), n, idx, nsrc, src, dst);
    return hip_check(hipGetLastError(), "gather_index");
}

int hx_scatter_index(int64_t n, const int64_t* idx, int64_t ndst, const double* src, double* dst, hx_stream stream) {
    if (n < 0 || ndst < 0 || (n > 0 && (!idx || !src || (ndst > 0 && !dst)))) {
        set_error("scatter_index: bad arguments");
        return HX_EINVAL;
    }
    if (n == 0) return HX_OK;
    const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(scatter_index, dim3(nb), dim3(256), 0, static_cast<hipStream_t>(stream), n, idx, ndst, src, dst);
    return hip_check(hipGetLastError(), "scatter_index");
}

int hx_axpy(int64_t n, double a, const double* x, double* y, hx_stream stream) {
    if (n < 0 || (n > 0 && (!x || !y))) {
        set_error("axpy: bad arguments");
        return HX_EINVAL;
    }
    if (n == 0) return HX_OK;
    const int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(axpy_f64, dim3(nb), dim3(256), 0, static_cast<hipStream_t>(stream), n, a, x, y);
    return hip_check(hipGetLastError(), "axpy");
}

int hx_heff_lower_f32(const hx_plan* plan, const double* L, const double* R, const void* ws, float* L32, float* R32,
                      void* ws32, hx_stream stream) {
    int rc = check_ready(plan, PK_HEFF, PK_HEFF_VJP);
    if (rc) return rc;
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if ((P->in_nnz && (!L || !L32)) || (P->in2_nnz && (!R || !R32)) || (P->ws_doubles && (!ws || !ws32))) {
        set_error("heff_lower_f32: null operand");
        return HX_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = cvt(P->in_nnz, L, L32, s))) return rc;
    if ((rc = cvt(P->in2_nnz, R, R32, s))) return rc;
    for (const auto& r : P->mix_ranges)
        if ((rc = cvt(r.second - r.first, static_cast<const double*>(ws) + r.first, static_cast<float*>(ws32) + r.first,
                      s)))
            return rc;
    if (P->kind == PK_HEFF_VJP && P->coef32_base >= 0 &&
        (rc = cvt((int64_t)P->coef.size(),
                  reinterpret_cast<const double*>(static_cast<const char*>(P->dev) + P->off_coef),
                  static_cast<float*>(ws32) + P->coef32_base, s)))
        return rc;
    return HX_OK;
}

extern "C++" {
template <bool BF>
static int apply_lowered(const hx_plan* plan, const float* L32, const float* R32, void* ws32, const float* psi32,
                         float* sigma32, hx_stream stream) {
    const char* what = BF ? "heff_apply_bf16" : "heff_apply_f32";
    int rc = check_ready(plan, PK_HEFF);
    if (rc) return rc;
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if ((P->psi_nnz && (!psi32 || !sigma32)) || (P->in_nnz && !L32) || (P->in2_nnz && !R32) ||
        (P->ws_doubles && !ws32)) {
        set_error(std::string(what) + ": null operand");
        return HX_EINVAL;
    }
    if (P->psi_nnz && psi32 == sigma32) {
        set_error(std::string(what) + ": psi and sigma must not alias");
        return HX_EINVAL;
    }
    BasesT<float> B{};
    B.p[SP_PSI] = const_cast<float*>(psi32);
    B.p[SP_OUT] = sigma32;
    B.p[SP_L] = const_cast<float*>(L32);
    B.p[SP_R] = const_cast<float*>(R32);
    B.p[SP_WS] = static_cast<float*>(ws32);
    B.p[SP_TAB] = nullptr;  // mixing (the only user of the coefficient table) runs in FP64
    B.p[SP_PART] = ws32 ? static_cast<float*>(ws32) + P->part_base : nullptr;
    for (const Launch& l : P->apply)
        if ((rc = launch_gemm<float, NSP_FWD, BF>(P, l, B, s_of(stream)))) return rc;
    return HX_OK;
}
}  // extern "C++"

int hx_heff_apply_f32(const hx_plan* plan, const float* L32, const float* R32, void* ws32, const float* psi32,
                      float* sigma32, hx_stream stream) {
    return apply_lowered<false>(plan, L32, R32, ws32, psi32, sigma32, stream);
}

int hx_heff_apply_bf16(const hx_plan* plan, const float* L32, const float* R32, void* ws32, const float* psi32,
                       float* sigma32, hx_stream stream) {
    return apply_lowered<true>(plan, L32, R32, ws32, psi32, sigma32, stream);
}

int hx_heff_diag(const hx_plan* plan, const double* L, const double* R, void* ws, double* diag, hx_stream stream) {
    int rc = check_ready(plan, PK_HEFF);
    if (rc) return rc;
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if ((P->psi_nnz && !diag) || (P->ws_doubles && !ws)) {
        set_error("heff_diag: null operand");
        return HX_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Bases B = make_bases(P, nullptr, diag, L, R, ws);
    for (const FillLaunch& f : P->diag_fill) {
        if (f.count <= 0) continue;
        int nb = (int)std::min<int64_t>(4096, (f.count + 255) / 256);
        hipLaunchKernelGGL(fill_zero<double>, dim3(nb), dim3(256), 0, s, B.p[f.space] + f.off, f.count);
        if ((rc = hip_check(hipGetLastError(), "diag fill"))) return rc;
    }
    const Gather* g = reinterpret_cast<const Gather*>(static_cast<const char*>(P->dev) + P->off_gathers);
    for (const GatherLaunch& gl : P->diag_gather) {
        hipLaunchKernelGGL(gather_scale<double>, dim3((unsigned)gl.ng), dim3(128), 0, s, g + gl.g0, B);
        if ((rc = hip_check(hipGetLastError(), "diag gather"))) return rc;
    }
    for (const Launch& l : P->diag_gemm)
        if ((rc = launch_gemm(P, l, B, s))) return rc;
    return HX_OK;
}

}  // extern "C"

// The backward launch sequence for FP64 or FP32 operands (FP32: environments, mixed
// operators and coefficient table lowered by hx_heff_lower_f32).
template <typename T>
static int backward_impl(const hx_plan* plan, const T* L, const T* R, void* ws, const T* psi, const T* g, T* g_psi,
                         T* g_L, T* g_R, T* g_W1, T* g_W2, hx_stream stream, const char* what) {
    int rc = check_ready(plan, PK_HEFF_VJP);
    if (rc) return rc;
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if ((P->psi_nnz && (!psi || !g || !g_psi)) || (P->in_nnz && (!L || !g_L)) || (P->in2_nnz && (!R || !g_R)) ||
        (P->w1_nnz && !g_W1) || (P->w2_nnz && !g_W2) || (P->ws_doubles && !ws)) {
        set_error(std::string(what) + ": null operand");
        return HX_EINVAL;
    }
    if (P->psi_nnz && (g_psi == psi || g_psi == g)) {
        set_error(std::string(what) + ": g_psi must not alias psi or g");
        return HX_EINVAL;
    }
    constexpr bool f64 = std::is_same<T, double>::value;
    if (!f64 && P->coef32_base < 0) {
        set_error(std::string(what) + ": plan has no FP32 coefficient table");
        return HX_EINVAL;
    }
    hipStream_t s = s_of(stream);
    T* w = static_cast<T*>(ws);
    BasesT<T> B{};
    B.p[SP_PSI] = const_cast<T*>(psi);
    B.p[SP_OUT] = g_psi;
    B.p[SP_L] = const_cast<T*>(L);
    B.p[SP_R] = const_cast<T*>(R);
    B.p[SP_WS] = w;
    B.p[SP_TAB] = f64 ? reinterpret_cast<T*>(static_cast<char*>(P->dev) + P->off_coef) : (w ? w + P->coef32_base : nullptr);
    B.p[SP_PART] = w ? w + P->part_base : nullptr;
    B.p[SP_G] = const_cast<T*>(g);
    B.p[SP_GL] = g_L;
    B.p[SP_GR] = g_R;
    B.p[SP_GW1] = g_W1;
    B.p[SP_GW2] = g_W2;
    for (const FillLaunch& f : P->bw_fill) {
        if (f.count <= 0) continue;
        int nb = (int)std::min<int64_t>(4096, (f.count + 255) / 256);
        hipLaunchKernelGGL(fill_zero<T>, dim3(nb), dim3(256), 0, s, B.p[f.space] + f.off, f.count);
        if ((rc = hip_check(hipGetLastError(), "backward fill"))) return rc;
    }
    const Gather* gt = reinterpret_cast<const Gather*>(static_cast<const char*>(P->dev) + P->off_gathers);
    for (const GatherLaunch& gl : P->bw_pre) {
        hipLaunchKernelGGL(copy_wide<T>, dim3((unsigned)gl.ng, 16), dim3(256), 0, s, gt + gl.g0, B);
        if ((rc = hip_check(hipGetLastError(), "backward staging copy"))) return rc;
    }
    for (const Launch& l : P->apply)
        if ((rc = launch_gemm<T, SP_N>(P, l, B, s))) return rc;
    for (const GatherLaunch& gl : P->bw_post) {
        hipLaunchKernelGGL(copy_wide<T>, dim3((unsigned)gl.ng, 16), dim3(256), 0, s, gt + gl.g0, B);
        if ((rc = hip_check(hipGetLastError(), "backward staging copy"))) return rc;
    }
    for (const GatherLaunch& gl : P->bw_gather) {
        hipLaunchKernelGGL(gather_scale<T>, dim3((unsigned)gl.ng), dim3(64), 0, s, gt + gl.g0, B);
        if ((rc = hip_check(hipGetLastError(), "backward gather"))) return rc;
    }
    return HX_OK;
}

extern "C" {

int hx_heff_apply_backward(const hx_plan* plan, const double* L, const double* R, void* ws, const double* psi,
                           const double* g, double* g_psi, double* g_L, double* g_R, double* g_W1, double* g_W2,
                           hx_stream stream) {
    return backward_impl<double>(plan, L, R, ws, psi, g, g_psi, g_L, g_R, g_W1, g_W2, stream,
                                 "heff_apply_backward");
}

int hx_heff_apply_backward_f32(const hx_plan* plan, const float* L32, const float* R32, void* ws32,
                               const float* psi32, const float* g32, float* g_psi32, float* g_L32, float* g_R32,
                               float* g_W1_32, float* g_W2_32, hx_stream stream) {
    return backward_impl<float>(plan, L32, R32, ws32, psi32, g32, g_psi32, g_L32, g_R32, g_W1_32, g_W2_32, stream,
                                "heff_apply_backward_f32");
}

int hx_env_update(const hx_plan* plan, const double* env_in, const double* site, void* ws, double* env_out,
                  hx_stream stream) {
    int rc = check_ready(plan, PK_ENV_LEFT);
    if (rc) return rc;
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if (P->kind == PK_HEFF) {
        set_error("env_update: plan is a sigma-vector plan");
        return HX_EINVAL;
    }
    if (!env_out || (P->in_nnz && !env_in) || (P->in2_nnz && !site) || (P->ws_doubles && !ws)) {
        set_error("env_update: null operand");
        return HX_EINVAL;
    }
    Bases B = make_bases(P, env_in, env_out, nullptr, site, ws);
    for (const Launch& l : P->apply)
        if ((rc = launch_gemm(P, l, B, static_cast<hipStream_t>(stream)))) return rc;
    return HX_OK;
}

int64_t hx_davidson_ws_bytes(int64_t n, int32_t kmax) {
    (void)n;
    (void)kmax;
    return DW_TOTAL * 8;
}

static int dots_into(int64_t n, int k, const double* a, int64_t lda, const double* b, double* ws, double* out,
                     int ostride, hipStream_t s) {
    hipLaunchKernelGGL(dots_pass1, dim3(DOT_BLOCKS), dim3(DOT_THREADS), 0, s, n, k, a, lda, b, ws + DW_P);
    hipLaunchKernelGGL(dots_pass2, dim3(1), dim3(DOT_BLOCKS), 0, s, k, ws + DW_P, out, ostride);
    return hip_check(hipGetLastError(), "dots");
}

int hx_dots(int64_t n, int32_t k, const double* a, int64_t lda, const double* b, void* ws, double* out,
            hx_stream stream) {
    if (k < 1 || k > KMAX || n < 0 || !a || !b || !ws || !out) {
        set_error("dots: bad arguments (1 <= k <= 32)");
        return HX_EINVAL;
    }
    return dots_into(n, k, a, lda, b, static_cast<double*>(ws), out, 1, static_cast<hipStream_t>(stream));
}

int hx_davidson_step(int64_t n, int32_t k, int32_t kmax, const double* V, int64_t ldv, const double* S, int64_t lds,
                     const double* diag, double guard, void* wsv, double* x, double* hx, double* t, double* scal,
                     hx_stream stream) {
    if (k < 1 || kmax > KMAX || k > kmax || n <= 0 || !V || !S || !diag || !wsv || !x || !hx || !t || !scal ||
        ldv < n || lds < n || !(guard > 0)) {
        set_error("davidson_step: bad arguments (1 <= k <= kmax <= 32, ld >= n, guard > 0)");
        return HX_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* ws = static_cast<double*>(wsv);
    int rc;
    const int kk = k - 1;
    // new column and row of G: G[i][kk] = v_i . s_kk, G[kk][i] = v_kk . s_i
    if ((rc = dots_into(n, k, V, ldv, S + (int64_t)kk * lds, ws, ws + DW_G + kk, KMAX, s))) return rc;
    if ((rc = dots_into(n, k, S, lds, V + (int64_t)kk * ldv, ws, ws + DW_G + (int64_t)kk * KMAX, 1, s))) return rc;
    hipLaunchKernelGGL(dav_eig, dim3(1), dim3(64), 0, s, k, ws, scal);
    if ((rc = hip_check(hipGetLastError(), "dav_eig"))) return rc;
    const int nb = (int)std::min<int64_t>(2048, (n + 255) / 256);
    hipLaunchKernelGGL(dav_combine, dim3(nb), dim3(256), 0, s, n, k, V, ldv, S, lds, ws, x, hx, t);
    if ((rc = hip_check(hipGetLastError(), "dav_combine"))) return rc;
    if ((rc = dots_into(n, 1, t, n, t, ws, ws + DW_S + 1, 1, s))) return rc;  // |r|^2
    hipLaunchKernelGGL(dav_precond, dim3(nb), dim3(256), 0, s, n, diag, guard, ws, t);
    if ((rc = hip_check(hipGetLastError(), "dav_precond"))) return rc;
    for (int pass = 0; pass < 2; ++pass) {
        if ((rc = dots_into(n, k, V, ldv, t, ws, ws + DW_C, 1, s))) return rc;
        hipLaunchKernelGGL(dav_project, dim3(nb), dim3(256), 0, s, n, k, V, ldv, ws, t);
        if ((rc = hip_check(hipGetLastError(), "dav_project"))) return rc;
    }
    if ((rc = dots_into(n, 1, t, n, t, ws, ws + DW_S + 2, 1, s))) return rc;  // |t|^2
    hipLaunchKernelGGL(dav_finish, dim3(nb), dim3(256), 0, s, n, ws, t, scal);
    return hip_check(hipGetLastError(), "dav_finish");
}

__global__ void scale_unit(int64_t n, double* __restrict__ x, const double* __restrict__ nrm2, double* norm_out) {
    const double nr = sqrt(nrm2[0]);
    const double inv = nr > 0 ? 1.0 / nr : 1.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        x[e] *= inv;
    if (blockIdx.x == 0 && threadIdx.x == 0 && norm_out) norm_out[0] = nr;
}

int hx_normalize(int64_t n, double* x, void* wsv, double* norm_out, hx_stream stream) {
    if (n <= 0 || !x || !wsv) {
        set_error("normalize: bad arguments");
        return HX_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* ws = static_cast<double*>(wsv);
    int rc;
    if ((rc = dots_into(n, 1, x, n, x, ws, ws + DW_S + 3, 1, s))) return rc;
    const int nb = (int)std::min<int64_t>(2048, (n + 255) / 256);
    hipLaunchKernelGGL(scale_unit, dim3(nb), dim3(256), 0, s, n, x, ws + DW_S + 3, norm_out);
    return hip_check(hipGetLastError(), "normalize");
}

int hx_davidson_restart2(int64_t n, const double* x, const double* hx, const double* xp, const double* hxp,
                         double* v1, double* s1, void* wsv, double* scal, hx_stream stream) {
    if (n <= 0 || !x || !hx || !xp || !hxp || !v1 || !s1 || !wsv || !scal) {
        set_error("davidson_restart2: bad arguments");
        return HX_EINVAL;
    }
    hipStream_t s = s_of(stream);
    double* ws = static_cast<double*>(wsv);
    const int nb = (int)std::min<int64_t>(2048, (n + 255) / 256);
    int rc;
    if ((rc = hip_check(hipMemcpyAsync(v1, xp, n * sizeof(double), hipMemcpyDeviceToDevice, s), "restart copy")) ||
        (rc = hip_check(hipMemcpyAsync(s1, hxp, n * sizeof(double), hipMemcpyDeviceToDevice, s), "restart copy")))
        return rc;
    for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
        if ((rc = dots_into(n, 1, x, n, v1, ws, ws + DW_S + 4, 1, s))) return rc;
        hipLaunchKernelGGL(restart_combine, dim3(nb), dim3(256), 0, s, n, x, hx, v1, s1, ws + DW_S + 4);
        if ((rc = hip_check(hipGetLastError(), "restart combine"))) return rc;
    }
    if ((rc = dots_into(n, 1, v1, n, v1, ws, ws + DW_S + 5, 1, s))) return rc;
    hipLaunchKernelGGL(restart_scale, dim3(nb), dim3(256), 0, s, n, v1, s1, ws + DW_S + 5, scal);
    return hip_check(hipGetLastError(), "restart scale");
}

// ---- HIP graphs of the sigma-vector launch sequence

struct hx_graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
};

int hx_heff_graph_create(const hx_plan* plan, int32_t what, const void* L, const void* R, void* ws, const void* psi,
                         void* sigma, hx_graph** out) {
    if (!out) {
        set_error("graph_create: null output");
        return HX_EINVAL;
    }
    *out = nullptr;
    if (what != HX_GRAPH_APPLY && what != HX_GRAPH_PREPARE_APPLY && what != HX_GRAPH_APPLY_F32 &&
        what != HX_GRAPH_APPLY_BF16) {
        set_error("graph_create: unknown sequence");
        return HX_EINVAL;
    }
    int rc = check_ready(plan, PK_HEFF);
    if (rc) return rc;
    hipStream_t cs;
    if ((rc = hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "graph_create: stream"))) return rc;
    if ((rc = hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "graph_create: begin capture"))) {
        (void)hipStreamDestroy(cs);
        return rc;
    }
    hx_stream hs = static_cast<hx_stream>(cs);
    if (what == HX_GRAPH_PREPARE_APPLY)
        rc = hx_heff_prepare(plan, static_cast<const double*>(L), static_cast<const double*>(R), ws, hs);
    if (rc == HX_OK && what == HX_GRAPH_APPLY_F32)
        rc = hx_heff_apply_f32(plan, static_cast<const float*>(L), static_cast<const float*>(R), ws,
                               static_cast<const float*>(psi), static_cast<float*>(sigma), hs);
    else if (rc == HX_OK && what == HX_GRAPH_APPLY_BF16)
        rc = hx_heff_apply_bf16(plan, static_cast<const float*>(L), static_cast<const float*>(R), ws,
                                static_cast<const float*>(psi), static_cast<float*>(sigma), hs);
    else if (rc == HX_OK)
        rc = hx_heff_apply(plan, static_cast<const double*>(L), static_cast<const double*>(R), ws,
                           static_cast<const double*>(psi), static_cast<double*>(sigma), hs);
    std::string saved = rc ? hx_last_error() : std::string();
    hipGraph_t g = nullptr;
    int rc2 = hip_check(hipStreamEndCapture(cs, &g), "graph_create: end capture");
    (void)hipStreamDestroy(cs);
    if (rc || rc2) {
        if (g) (void)hipGraphDestroy(g);
        if (rc) set_error(saved);
        return rc ? rc : rc2;
    }
    hx_graph* G = new hx_graph();
    G->g = g;
    if ((rc = hip_check(hipGraphInstantiate(&G->e, g, nullptr, nullptr, 0), "graph_create: instantiate"))) {
        (void)hipGraphDestroy(g);
        delete G;
        return rc;
    }
    *out = G;
    return HX_OK;
}

int hx_graph_launch(hx_graph* graph, hx_stream stream) {
    if (!graph || !graph->e) {
        set_error("graph_launch: null graph");
        return HX_EINVAL;
    }
    return hip_check(hipGraphLaunch(graph->e, s_of(stream)), "graph_launch");
}

void hx_graph_destroy(hx_graph* graph) {
    if (!graph) return;
    if (graph->e) (void)hipGraphExecDestroy(graph->e);
    if (graph->g) (void)hipGraphDestroy(graph->g);
    delete graph;
}

}  // extern "C"

// ---------------------------------------------------------------- no-allocation sigma-vector
//
// hx_heff_apply_noalloc: prepare + apply with the workspace in a fixed device array of
// this file instead of a caller buffer, for callers that cannot allocate.  The array
// is a device symbol: its host-side name is not a device address, so the address is
// taken once per device with hipGetSymbolAddress and only that address reaches the
// kernels.

static __device__ __align__(256) double scratch[HX_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the scratch array on the current device (looked up on the first
// call on that device).
static int scratch_on_current_device(void** out) {
    int dev = -1;
    int rc = hip_check(hipGetDevice(&dev), "heff_apply_noalloc: current device");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("heff_apply_noalloc: device index out of range");
        return HX_EUNSUP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if ((rc = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "heff_apply_noalloc: scratch address")))
            return rc;
        if (!ptr) {
            set_error("heff_apply_noalloc: scratch address is null");
            return HX_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HX_OK;
}

extern "C" {

int hx_heff_apply_noalloc(const hx_plan* plan, const double* L, const double* R, const double* psi, double* sigma,
                          hx_stream stream) {
    if (!plan) {
        set_error("heff_apply_noalloc: null plan");
        return HX_EINVAL;
    }
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if (P->kind != PK_HEFF) {
        set_error("heff_apply_noalloc: needs a sigma-vector plan");
        return HX_EINVAL;
    }
    const int64_t need = P->ws_doubles * (int64_t)sizeof(double);
    if (need > (int64_t)HX_NOALLOC_SCRATCH_BYTES) {
        set_error("heff_apply_noalloc: the plan's workspace (" + std::to_string(need) +
                  " bytes) exceeds the static scratch of " + std::to_string((long long)HX_NOALLOC_SCRATCH_BYTES) +
                  " bytes (use hx_heff_prepare + hx_heff_apply with a caller workspace)");
        return HX_EINVAL;
    }
    int rc = check_ready(plan, PK_HEFF);
    if (rc) return rc;
    if ((P->psi_nnz && (!psi || !sigma)) || (P->in_nnz && !L) || (P->in2_nnz && !R)) {
        set_error("heff_apply_noalloc: null operand");
        return HX_EINVAL;
    }
    if (P->psi_nnz && psi == sigma) {
        set_error("heff_apply_noalloc: psi and sigma must not alias");
        return HX_EINVAL;
    }
    void* ws = nullptr;
    if ((rc = scratch_on_current_device(&ws))) return rc;
    // every region of the workspace (mixed operators, intermediates, split-K partials)
    // is written before it is read within this call: nothing needs clearing
    hipStream_t s = s_of(stream);
    Bases B = make_bases(P, psi, sigma, L, R, ws);
    if ((rc = run_prepare(P, B, s))) return rc;
    for (const Launch& l : P->apply)
        if ((rc = launch_gemm(P, l, B, s))) return rc;
    return HX_OK;
}

}  // extern "C"
