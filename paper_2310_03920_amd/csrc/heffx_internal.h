// Internal tables shared by the host plan builder and the gfx950 kernels.
#pragma once
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

namespace hx {

// Operand spaces: a task names its operands as (space, element offset); the
// launcher passes one base pointer per space, so a plan is independent of the
// buffers it is applied to.
enum Space : int8_t {
    SP_PSI = 0,   // input vector (psi) / input environment for env updates
    SP_OUT = 1,   // output (sigma / updated environment / diag)
    SP_L = 2,     // left environment payload
    SP_R = 3,     // right environment payload (env update: site tensor)
    SP_WS = 4,    // caller workspace (mixed operators, intermediates)
    SP_TAB = 5,   // plan tables on the device (mixing coefficients)
    SP_PART = 6,  // split-K partial tiles (a region of the workspace)
    SP_G = 7,     // adjoint: cotangent of sigma (wavefunction layout)
    SP_GL = 8,    // adjoint: gradient of the left environment payload
    SP_GR = 9,    // adjoint: gradient of the right environment payload
    SP_GW1 = 10,  // adjoint: gradient of the values of W1 (16 per MPO entry)
    SP_GW2 = 11,  // adjoint: gradient of the values of W2
    SP_N = 12
};

// One contribution alpha * op(A) * op(B) to an output tile.  A is (rows x k),
// B is (k x cols); with TRANS the stored matrix is the transpose.  For a tile
// at (r0, c0) inside its block the kernel offsets A by r0 rows and B by c0 cols.
struct Task {
    int64_t aoff;
    int64_t boff;
    int32_t lda;
    int32_t ldb;
    int32_t k;
    int32_t spaces;   // aspace | bspace << 8 (one dword: read with scalar loads)
    double alpha;
    int aspace() const { return spaces & 0xff; }
    int bspace() const { return (spaces >> 8) & 0xff; }
    void set_spaces(int a, int b) { spaces = (a & 0xff) | ((b & 0xff) << 8); }
};
static_assert(sizeof(Task) == 40, "Task layout");

// One output tile (at most TM x TN) of one output block.
struct Tile {
    int64_t coff;     // element offset of the tile's first element in cspace
    int32_t ldc;
    int32_t m, n;     // tile extent
    int32_t r0, c0;   // tile origin inside its block
    int32_t tbeg;     // task range [tbeg, tend)
    int32_t tend;
    int32_t ktot;     // sum over the task range of k rounded up to a multiple of 16
    int32_t flags;    // cspace | beta << 8
    int cspace() const { return flags & 0xff; }
    int beta() const { return (flags >> 8) & 0xff; }
    void set_out(int space, int b) { flags = (space & 0xff) | ((b & 0xff) << 8); }
};
static_assert(sizeof(Tile) == 48, "Tile layout");

// Strided copy with scale: dst[d + x*ds] = alpha * src[s + x*ss], x < count.
struct Gather {
    int64_t soff;
    int64_t doff;
    int32_t sstride;
    int32_t dstride;
    int32_t count;
    int8_t sspace;
    int8_t dspace;
    int16_t pad;
    double alpha;
};
static_assert(sizeof(Gather) == 40, "Gather layout");

// Fixed-order sum of a split tile's partials: out = beta*out + sum_j part[j].
struct Reduce {
    int64_t coff;     // output tile (cspace)
    int64_t pbase;    // first partial (SP_PART), partial j at pbase + j*TM*TN, ld TN
    int32_t ldc;
    int32_t m, n;
    int32_t np;
    int8_t cspace;
    int8_t beta;
    int16_t pad;
    int32_t pld;      // leading dimension of the partial tiles (the launch's tile columns)
};
static_assert(sizeof(Reduce) == 40, "Reduce layout");

// Tile shapes (4 waves of 32 x 32 each): 64 x 64, 128 x 32 (narrow blocks), 32 x 128
// (short blocks); and 32 x 32 computed by a single wave (blocks of at most 32 x 32).
// A split-K partial slot holds TM * TN elements, enough for every shape.
constexpr int TM = 64;
constexpr int TN = 64;
enum TileShape : int { SH_SQ = 0, SH_TALL = 1, SH_WIDE = 2, SH_SMALL = 3 };
inline int shape_rows(int sh) { return sh == SH_TALL ? 128 : (sh == SH_WIDE || sh == SH_SMALL) ? 32 : 64; }
inline int shape_cols(int sh) { return sh == SH_WIDE ? 128 : (sh == SH_TALL || sh == SH_SMALL) ? 32 : 64; }

enum TransKind : int { NN = 0, NT = 1, TN_ = 2 };

// A GEMM launch: tiles [tile0, tile0+ntile) and their tasks in the device table.
struct Launch {
    int kind;          // TransKind
    int shape = SH_SQ; // TileShape of every tile of the launch
    int stage = 0;     // which round of the plan produced it (launches of one stage are independent)
    int64_t tile0;     // index into the plan's tile array
    int64_t ntile;
    double flops;      // algorithmic 2 m n k of the blocks it covers
    int64_t red0 = 0;  // split-K reductions run after the GEMM: [red0, red0+nred)
    int64_t nred = 0;
};

struct GatherLaunch {
    int64_t g0, ng;
};

struct FillLaunch {
    int8_t space;
    int64_t off, count;
};

enum PlanKind : int { PK_HEFF = 0, PK_ENV_LEFT = 1, PK_ENV_RIGHT = 2, PK_HEFF_VJP = 3 };

struct Plan {
    int kind = PK_HEFF;
    // host tables (uploaded into one device buffer)
    std::vector<Tile> tiles;
    std::vector<Task> tasks;
    std::vector<Gather> gathers;
    std::vector<Reduce> reduces;
    std::vector<double> coef;     // mixing coefficient matrices (space SP_TAB)
    // sequences of launches
    std::vector<Launch> prep;     // mixing (heff_prepare / first part of env update)
    std::vector<GatherLaunch> prep_gather;  // after the mixing: stacked first-round operands
    std::vector<Launch> apply;    // sigma (heff) or E1/E2 chunks (env)
    std::vector<FillLaunch> diag_fill;
    std::vector<GatherLaunch> diag_gather;
    std::vector<Launch> diag_gemm;
    // adjoint plans: zero fills before, coefficient-gradient gathers after the GEMM launches
    std::vector<FillLaunch> bw_fill;
    std::vector<GatherLaunch> bw_gather;
    // adjoint plans: whole-payload copies before (bw_pre) and after (bw_post) the GEMM
    // launches (environment operators of one shift class staged contiguously)
    std::vector<GatherLaunch> bw_pre, bw_post;
    int64_t w1_nnz = 0, w2_nnz = 0;  // MPO entries of the two sites (gradient lengths / 16)
    // sizes
    int64_t psi_nnz = 0, in_nnz = 0, in2_nnz = 0, out_nnz = 0;
    int64_t ws_doubles = 0;
    int64_t part_base = 0;      // workspace offset (doubles) of the split-K partial region
    int64_t coef32_base = -1;   // adjoint plans: FP32 copy of the coefficient table (workspace elements)
    int64_t mix_end = 0;        // workspace elements [0, mix_end) hold the mixed operators
    std::vector<std::pair<int64_t, int64_t>> mix_ranges;  // batched plans: per-instance mixed ranges
    // batched plans: per-instance element offsets of psi/sigma, L, R in the concatenated buffers
    std::vector<int64_t> inst_psi, inst_L, inst_R;
    int64_t part_tiles = 0;     // partial tiles needed by the largest launch
    // tile ranges [first, first + count) of launches whose XCD ordering is still to be
    // done (the ranges are disjoint; they are ordered on host threads before packing)
    std::vector<std::pair<int64_t, int64_t>> sort_ranges;
    int64_t split_kseg_min = 2048;
    int variant = 0;            // block-GEMM pipeline variant (see hx_plan_opts.kernel_variant)
    int kstage = 16;            // K-stage depth of that variant; task K is padded to it
    int n_roots = 1;            // vectors per sigma-vector call (roots side by side in column blocks)
    int b_part = 0, b_nparts = 1;  // sigma-vector plans: only middle-bond indices b = b_part (mod b_nparts)
    bool t_merge = true;        // sigma-vector plans: merge first-round intermediates with equal psi-side tasks
    int n_stages = 0;           // rounds emitted so far (Launch::stage)
    double flops_apply = 0, flops_prepare = 0, bytes_apply = 0;
    double flops_useful = -1;   // sigma plans: block-product work whose results sigma reads (< 0: = flops_apply)
    int64_t n_tasks_apply = 0, n_tiles_apply = 0;
    int n_chunks = 0, n_mixed = 0;
    // device table layout (byte offsets inside the uploaded buffer)
    int64_t off_tiles = 0, off_tasks = 0, off_gathers = 0, off_coef = 0, off_reduces = 0, table_bytes = 0;
    void* dev = nullptr;          // caller-provided device table buffer (after upload)
};

void set_error(const std::string& msg);

}  // namespace hx
