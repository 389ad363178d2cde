/*
 * heffx -- MI355X (gfx950) library for the two-site DMRG sigma-vector path of an
 * ab initio Hamiltonian with U(1) x U(1) (particle number N, 2*Sz) symmetry.
 *
 * The operation (Sec. II.A.2 two-site sweep; Sec. II.C.1 NC-partition MPO whose
 * bond operators are the normal / complementary renormalised operators):
 *
 *   sigma[l',s1',s2',r'] = sum_{a,b,c} sum_{l,s1,s2,r}
 *       L_a[l',l] W1_ab[s1',s1] W2_bc[s2',s2] R_c[r',r] psi[l,s1,s2,r]
 *
 * with L_a / R_c the left / right environment operators (block-sparse by
 * symmetry sector, Sec. II.A.1), W1 / W2 the MPO tensors of the two sites whose
 * 4x4 site matrices already carry the Jordan-Wigner parity strings, so every
 * product is a plain Kronecker product.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Site basis: [empty, alpha, beta, alpha-beta], (N, 2Sz) = (0,0),(1,1),(1,-1),(2,0)
 * (Listing 1).  A bond is labelled by the quantum number of its LEFT block.
 * A bond table lists sectors sorted lexicographically by (N, 2Sz).
 * An operator set lists, per operator, the shift dq = (dN, d2Sz) it applies to
 * the left-block label of the sectors it acts on (for a right-environment
 * operator this is the shift on the same left-block labels of its bond).
 *
 * Payload layouts (FP64, all blocks row-major, no padding):
 *  - environment: operators in order; operator a holds one block per source
 *    sector q (ascending) whose destination q+dq_a exists; block (dst x src).
 *  - two-site wavefunction between bond i and bond i+2: column blocks
 *    (s2, ir) ascending; inside one, the row blocks (il, s1) ascending with
 *    q(il)+q(s1)+q(s2) = q(ir); block (dim il x dim ir).  A column block is
 *    thus one dense row-major matrix (sum of dim il) x dim ir.
 *  - site tensor between bond k and k+1: blocks for (il, s) ascending whose right
 *    sector q(il)+q(s) exists; block (dim il x dim ir).
 * The hx_*_layout functions return these offsets.
 *
 * Memory: the library never allocates device memory.  Plans are built on the
 * host (no HIP call); the caller allocates the device table buffer and the
 * workspace with the sizes reported by hx_plan_get_info and passes them in.  All
 * device calls are asynchronous on the caller's stream.
 *
 * Errors: every int-returning call returns 0 on success, HX_EINVAL for a
 * malformed table or argument (and, from the plan builders, for host memory
 * exhausted while building), HX_EHIP for a HIP failure, HX_EUNSUP for an
 * unsupported request; hx_last_error() returns a thread-local message.  A device
 * buffer may be NULL exactly when the plan gives it length zero (e.g. psi and
 * sigma of a two-site space with no allowed block: the call is then a no-op).
 */
#ifndef HEFFX_H
#define HEFFX_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HX_OK 0
#define HX_EINVAL (-1)
#define HX_EHIP (-2)
#define HX_EUNSUP (-3)

typedef struct hx_plan hx_plan;
typedef void* hx_stream; /* hipStream_t of the caller (0 = null stream) */

/* Sector table of one bond: nsec sectors; qn[2*i] = N, qn[2*i+1] = 2Sz; dim[i] > 0. */
typedef struct {
    int32_t nsec;
    const int32_t* qn;
    const int32_t* dim;
} hx_bond;

/* Operator set: nop operators, dq[2*a] = dN, dq[2*a+1] = d2Sz. */
typedef struct {
    int32_t nop;
    const int32_t* dq;
} hx_opset;

/* MPO tensor of one site in coordinate form: entry e couples operator row[e] of
 * the cut on its left to operator col[e] of the cut on its right with the 4x4
 * site matrix val[16*e + 4*s_out + s_in].  Entries need not be sorted; repeated
 * (row, col) pairs are summed.  Each site matrix must shift the site quantum
 * number by exactly dq(col) - dq(row); other elements must be zero. */
typedef struct {
    int64_t nnz;
    const int32_t* row;
    const int32_t* col;
    const double* val;
} hx_mpo_site;

typedef struct {
    int64_t t_budget_bytes;  /* cap on the intermediate (T) workspace; 0 = default 1 GiB */
    int32_t split_kseg_min;  /* minimum K of a split-K segment; 0 = default 2048 */
    int32_t kernel_variant;  /* block-GEMM pipeline: 0 = two LDS buffers, 16-deep K stages (default);
                                1 = one LDS buffer, 16-deep (more workgroups per CU);
                                2 = two LDS buffers, 8-deep (less K padding, more workgroups per CU);
                                3 = removed (persistent workgroups; rejected with HX_EINVAL);
                                4, 5 = as 0, 1 with 128 x 32 tiles for narrow and 32 x 128 tiles for
                                short blocks (one launch per tile shape);
                                6 = as 1 with single-wave 32 x 32 tiles for blocks of at most
                                32 x 32 (FP64 / FP32; BF16 products: HX_EUNSUP).
                                Results are identical up to FP rounding order of the padding. */
    int32_t n_roots;         /* sigma-vector plans: number of vectors R applied per call (0 = 1, at
                                most 64; the state-averaged multi-root form of Sec. II.A.3).  psi and
                                sigma then hold, in every column block (s2, ir), the R roots side by
                                side: element (row, rho, r) at R*off + row*R*dim(ir) + rho*dim(ir) + r,
                                off = the single-root offset of the column block; the second GEMM
                                round runs on R times the columns.  diag stays single-root.  Adjoint
                                plans need R = 1. */
    int32_t b_part;
    int32_t b_nparts;        /* sigma-vector plans: with b_nparts > 1 the plan keeps only the terms of
                                the middle-bond operators b with b mod b_nparts == b_part (the MPO
                                column / row index shared by W1 and W2): prepare, apply and diag
                                give that part's share, and the shares of the b_nparts parts sum to
                                the whole -- the split of the sigma-vector over the paper's normal
                                and complementary operators (Sec. II.B.1 (iii)) that several GPUs
                                would each take one part of, with one sum of sigma afterwards.
                                b_nparts 0 or 1 (and b_part 0) = all operators.  Other plan kinds:
                                HX_EUNSUP for b_nparts > 1; HX_EINVAL for b_part outside
                                [0, b_nparts). */
    int32_t t_merge_off;     /* sigma-vector plans: nonzero keeps one first-round intermediate per middle
                                operator b.  By default (0) the intermediates T_b that share their
                                whole first-round task list on the psi side (same psi rows, same
                                contraction lengths; single-root plans) are laid side by side as one
                                wide matrix, and the right mixed operators they multiply are copied,
                                scaled by their coefficients, into one stacked operand per task at
                                hx_heff_prepare, so one GEMM with full-width tiles replaces many narrow
                                ones.  The workspace grows by the stacked copies; results differ only
                                in rounding. */
    int32_t reserved[2];
} hx_plan_opts;

typedef struct {
    int64_t psi_nnz;        /* wavefunction / sigma length (doubles) */
    int64_t in_nnz;         /* heff: left-env payload length; env: input env payload */
    int64_t in2_nnz;        /* heff: right-env payload length; env: site tensor payload */
    int64_t out_nnz;        /* env: output env payload length; heff: 0 */
    int64_t table_bytes;    /* device table buffer the caller provides to hx_plan_upload */
    int64_t ws_bytes;       /* workspace the caller provides to prepare/apply/update */
    double flops_apply;     /* algorithmic FLOP of one hx_heff_apply or hx_env_update */
    double flops_prepare;   /* algorithmic FLOP of operator mixing (hx_heff_prepare) */
    double bytes_apply;     /* algorithmic operand bytes of one apply (each operand block once) */
    int64_t n_tasks;        /* GEMM tasks of one apply */
    int64_t n_tiles;        /* output tiles of one apply */
    int32_t n_chunks;       /* number of intermediate chunks */
    int32_t n_mixed;        /* number of materialised mixed operators */
    double flops_useful;    /* sigma-vector plans: the part of flops_apply whose results sigma
                               reads (a stacked stage-1 intermediate is computed over the span
                               of rows stage 2 reads, which may enclose rows it does not read);
                               other plans: flops_apply */
} hx_plan_info;

/* ---- layouts (host only) ---------------------------------------------------- */

/* Environment payload offsets: op_off[nop+1] (op a occupies [op_off[a], op_off[a+1]));
 * blk_off[nop*nsec] = offset of the block with source sector q, or -1. */
int hx_env_layout(const hx_bond* bond, const hx_opset* ops, int64_t* op_off, int64_t* blk_off);

/* Two-site wavefunction layout: writes up to max_blocks keys (il,s1,s2,ir as 4
 * int32 each) and offsets (max_blocks+1 entries incl. the total); returns the
 * number of blocks or a negative error. keys/off may be NULL to query the count. */
int64_t hx_psi_layout(const hx_bond* lbond, const hx_bond* rbond, int64_t max_blocks,
                      int32_t* keys, int64_t* off);

/* Site tensor layout: keys (il, s, ir) as 3 int32 each; same rules as hx_psi_layout. */
int64_t hx_site_layout(const hx_bond* lbond, const hx_bond* rbond, int64_t max_blocks,
                       int32_t* keys, int64_t* off);

/* ---- sigma-vector plan ------------------------------------------------------ */

/* Build (host only) the plan of sigma = H_eff psi for the two-site step between
 * bond lbond (left environment Lops acting on it) and bond rbond (right
 * environment Rops), with W1 coupling Lops -> mid and W2 coupling mid -> Rops.
 * Validates every table; rejects shifts that break quantum-number conservation. */
int hx_heff_plan_create(const hx_bond* lbond, const hx_bond* rbond, const hx_opset* Lops,
                        const hx_opset* mid, const hx_opset* Rops, const hx_mpo_site* W1,
                        const hx_mpo_site* W2, const hx_plan_opts* opts, hx_plan** out);

/* Build (host only) the plan of an environment update (Sec. II.A.2 sweep):
 *  direction 0 (left, L -> R):  L'_b = sum_{a,s,t} A[.,s,.]^T (L_a W_ab[s,t]) A[.,t,.]
 *     bond_in = bond k, bond_out = bond k+1, ops_in at cut k, ops_out at cut k+1,
 *     W = MPO of site k (rows ops_in, cols ops_out), site tensor A between bond_in and bond_out.
 *  direction 1 (right, R -> L): R'_a = sum_{b,s,t} B[.,s,.] (W_ab[s,t] R_b) B[.,t,.]^T
 *     bond_in = bond k+1, bond_out = bond k, ops_in at cut k+1, ops_out at cut k,
 *     W = MPO of site k (rows ops_out, cols ops_in), site tensor B between bond_out and bond_in. */
int hx_env_plan_create(int direction, const hx_bond* bond_in, const hx_bond* bond_out,
                       const hx_opset* ops_in, const hx_opset* ops_out, const hx_mpo_site* W,
                       const hx_plan_opts* opts, hx_plan** out);

int hx_plan_get_info(const hx_plan* plan, hx_plan_info* info);

/* Copy the plan's tables to caller memory `dev_tables` (table_bytes, 256-byte
 * aligned device memory).  Must precede every device call with this plan. */
int hx_plan_upload(hx_plan* plan, void* dev_tables, hx_stream stream);

void hx_plan_destroy(hx_plan* plan);

/* Mixed operators sum_a W1_ab[s1',s1] L_a and sum_c W2_bc[s2',s2] R_c into ws
 * (Sec. II.C.1 integral-weighted sums building the complementary operators).
 * Needed once per (L, R) before hx_heff_apply / hx_heff_diag. */
int hx_heff_prepare(const hx_plan* plan, const double* L, const double* R, void* ws,
                    hx_stream stream);

/* sigma = H_eff psi (sigma overwritten).  ws must hold the result of
 * hx_heff_prepare for the same L and R.  psi and sigma must not overlap. */
int hx_heff_apply(const hx_plan* plan, const double* L, const double* R, void* ws,
                  const double* psi, double* sigma, hx_stream stream);

/* diag = diagonal of H_eff in the wavefunction layout (ws prepared as above). */
int hx_heff_diag(const hx_plan* plan, const double* L, const double* R, void* ws,
                 double* diag, hx_stream stream);

/* env_out = updated environment (overwritten); see hx_env_plan_create. */
int hx_env_update(const hx_plan* plan, const double* env_in, const double* site, void* ws,
                  double* env_out, hx_stream stream);

/* ---- one-site sweep ---------------------------------------------------------- */

/* One-site wavefunction layout (the one-site sweep of Sec. II.A.2): column blocks ir
 * ascending; inside one, row blocks (il, s) ascending with q(il) + q(s) = q(ir);
 * block (dim il x dim ir) row-major.  keys: (il, s, ir) as 3 int32; otherwise as
 * hx_psi_layout. */
int64_t hx_psi1_layout(const hx_bond* lbond, const hx_bond* rbond, int64_t max_blocks,
                       int32_t* keys, int64_t* off);

/* Plan of the one-site sigma = sum_{a,b} L_a (x) W_ab (x) R_b psi between bond lbond
 * (left environment Lops) and bond rbond (right environment Rops), W the MPO tensor of
 * the site (rows Lops, cols Rops).  Used with hx_plan_get_info / upload / destroy,
 * hx_heff_prepare, hx_heff_apply, hx_heff_diag, the FP32/BF16 entry points and graphs,
 * exactly as a two-site plan, with psi in the hx_psi1_layout layout.  Same kernels:
 * the absent second site makes the right mixed operators the R_b themselves. */
int hx_heff1_plan_create(const hx_bond* lbond, const hx_bond* rbond, const hx_opset* Lops,
                         const hx_opset* Rops, const hx_mpo_site* W, const hx_plan_opts* opts,
                         hx_plan** out);

/* ---- adjoint (vector-Jacobian products of the sigma-vector) ----------------- */

/* Build (host only) the plan of the VJP of sigma = H_eff(L, W1, W2, R) psi, same
 * arguments as hx_heff_plan_create.  Given a cotangent g (the gradient of a
 * scalar f with respect to sigma, wavefunction layout) it yields df/dpsi, df/dL,
 * df/dR and df/dW1, df/dW2.  With g = psi these are the derivatives of
 * <psi|H_eff|psi> with respect to L, W and R (the quantities from which reduced
 * density matrices and integral gradients follow, Sec. II.E.1 and the
 * DMRG-CASSCF gradients of Sec. II.A.8), and df/dpsi + H_eff psi is its psi
 * gradient.
 * The plan's hx_plan_get_info reports the backward FLOP as flops_apply. */
int hx_heff_vjp_plan_create(const hx_bond* lbond, const hx_bond* rbond, const hx_opset* Lops,
                            const hx_opset* mid, const hx_opset* Rops, const hx_mpo_site* W1,
                            const hx_mpo_site* W2, const hx_plan_opts* opts, hx_plan** out);

/* VJP plan of the one-site sigma-vector (arguments as hx_heff1_plan_create): used
 * with hx_heff_prepare / hx_heff_apply_backward like a two-site VJP plan, psi and g
 * in the hx_psi1_layout layout; g_W1 is the gradient of W's values, g_W2 (16 x the
 * number of Rops operators) belongs to the identity coupling on the absent site and
 * carries no information.  Environment updates are adjoints of this form: for a
 * left update L'_b = sum_{a,s',s} W_ab[s',s] A_s'^T L_a A_s and a cotangent G of L',
 * <G, L'> = <A, H1(L, W, R := G) A> (the same holds for right updates with G as the
 * left environment), so with psi = g = A this plan gives d<G,L'>/dL (g_L),
 * d<G,L'>/dW (g_W1) and, with H1 A from the forward plan, d<G,L'>/dA =
 * H1 A + H1^T A -- the chain through hx_env_update of Sec. II.E.1 gradients. */
int hx_heff1_vjp_plan_create(const hx_bond* lbond, const hx_bond* rbond, const hx_opset* Lops,
                             const hx_opset* Rops, const hx_mpo_site* W, const hx_plan_opts* opts,
                             hx_plan** out);

/* Backward of hx_heff_apply with an uploaded VJP plan whose workspace holds
 * hx_heff_prepare(plan, L, R, ws) for the same L and R.  Outputs (overwritten,
 * device, FP64):
 *   g_psi  (psi_nnz)   = H_eff^T g                       (wavefunction layout)
 *   g_L    (in_nnz)    = df/dL, left-environment payload layout
 *   g_R    (in2_nnz)   = df/dR, right-environment payload layout
 *   g_W1   (16 x W1->nnz), g_W2 (16 x W2->nnz): df/dval for every NONZERO site-
 *          matrix value of the MPO tables passed at plan creation, in their
 *          val[] layout; entries whose value is zero are written as 0.
 * The operation is the exact transpose of the forward contraction in the
 * forward's block structure (Sec. II.C.1 operator mixing, both GEMM rounds).
 * g_psi must not alias psi or g.  Deterministic: no atomics, fixed order. */
int hx_heff_apply_backward(const hx_plan* plan, const double* L, const double* R, void* ws,
                           const double* psi, const double* g, double* g_psi, double* g_L,
                           double* g_R, double* g_W1, double* g_W2, hx_stream stream);

/* hx_heff_apply_backward with FP32 operands and FP32 MFMA accumulation: L32, R32 and
 * ws32 from hx_heff_lower_f32 on the VJP plan (after hx_heff_prepare in FP64), psi32
 * and g32 in FP32, all outputs FP32 in the layouts of hx_heff_apply_backward.  The
 * precision mode of the gradients (the FP32 case of the differentiation
 * configuration); relative error ~1e-6 of the operands' scale. */
int hx_heff_apply_backward_f32(const hx_plan* plan, const float* L32, const float* R32, void* ws32,
                               const float* psi32, const float* g32, float* g_psi32, float* g_L32,
                               float* g_R32, float* g_W1_32, float* g_W2_32, hx_stream stream);

/* ---- batching: many independent sigma-vector problems per launch ----------- */

/* Merge n sigma-vector plans (each built by hx_heff_plan_create; HX_EUNSUP for
 * other plan kinds) into one plan whose prepare, apply and diag stages issue
 * their launches round by round: the k-th launch of the merged sequence covers
 * the next launch of every instance that has one (of the same GEMM form and
 * tile shape).  Single-chunk instances give the same number of launches as ONE
 * instance, each covering all instances; an instance split into several
 * intermediate chunks takes part in as many rounds as its own sequence has, so
 * a small budget per instance keeps each round's intermediates small.
 * This is the data parallelism across independent two-site problems (several
 * states, sites or molecules) that the sweep of Sec. II.A.2 does not expose
 * within one step.  Instance i's operands are placed in concatenated buffers:
 * psi/sigma/diag at psi_off(i), L at L_off(i), R at R_off(i) (elements, from
 * hx_batch_offsets); the workspace and tables are the merged plan's own.  The
 * merged plan is used with the ordinary entry points (prepare, apply, diag,
 * lower_f32, apply_f32); each instance's sigma equals, bit for bit, what its
 * own plan produces.  The input plans are not modified and may be destroyed. */
int hx_heff_plan_batch(const hx_plan* const* plans, int32_t n, hx_plan** out);

/* Element offsets of instance i inside the concatenated psi/sigma, L and R
 * buffers of a batched plan (any pointer may be NULL).  HX_EINVAL if the plan
 * is not batched or i is out of range. */
int hx_batch_offsets(const hx_plan* plan, int32_t i, int64_t* psi_off, int64_t* L_off, int64_t* R_off);

/* ---- HIP graphs ------------------------------------------------------------ */

typedef struct hx_graph hx_graph;

#define HX_GRAPH_APPLY 1          /* hx_heff_apply (FP64 pointers) */
#define HX_GRAPH_PREPARE_APPLY 2  /* hx_heff_prepare then hx_heff_apply (FP64 pointers) */
#define HX_GRAPH_APPLY_F32 3      /* hx_heff_apply_f32 (L32, R32, ws32, psi32, sigma32) */
#define HX_GRAPH_APPLY_BF16 4     /* hx_heff_apply_bf16 (same operands as HX_GRAPH_APPLY_F32) */

/* Capture the launch sequence `what` of an uploaded sigma-vector plan (single
 * or batched) with these operand pointers into an executable HIP graph, so one
 * hx_graph_launch replays every launch of the step.  The pointers are baked into
 * the graph: they must stay valid, and their contents are read / written at
 * each launch.  The sequences contain kernel launches only (no memset or copy
 * nodes).  Capture uses a private stream and runs nothing; HIP allocates the
 * graph's own host/device bookkeeping, released by hx_graph_destroy. */
int hx_heff_graph_create(const hx_plan* plan, int32_t what, const void* L, const void* R, void* ws,
                         const void* psi, void* sigma, hx_graph** out);

/* Enqueue one replay of the graph on `stream` (asynchronous). */
int hx_graph_launch(hx_graph* graph, hx_stream stream);

void hx_graph_destroy(hx_graph* graph);

/* ---- FP32 precision mode (the Davidson work stays FP64) -------------------- */

/* Element-wise conversions (n elements, device pointers). */
int hx_convert_f64_f32(int64_t n, const double* src, float* dst, hx_stream stream);
int hx_convert_f32_f64(int64_t n, const float* src, double* dst, hx_stream stream);

/* Element moves between payload layouts (e.g. a site tensor, hx_site_layout, and the
 * same tensor as a one-site wavefunction, hx_psi1_layout):
 *   hx_gather_index : dst[j] = src[idx[j]]   for j < n
 *   hx_scatter_index: dst[idx[j]] = src[j]   for j < n
 * idx: n int64 on the device (caller-owned); an index outside [0, nsrc) resp.
 * [0, ndst) leaves its element unchanged.  hx_axpy: y += a x over n doubles.  All
 * device, asynchronous on the stream; HX_EINVAL for negative sizes or NULL buffers
 * of nonzero length. */
int hx_gather_index(int64_t n, const int64_t* idx, int64_t nsrc, const double* src, double* dst,
                    hx_stream stream);
int hx_scatter_index(int64_t n, const int64_t* idx, int64_t ndst, const double* src, double* dst,
                     hx_stream stream);
int hx_axpy(int64_t n, double a, const double* x, double* y, hx_stream stream);

/* Round the operands of a prepared sigma-vector plan to FP32: L -> L32 (in_nnz
 * floats), R -> R32 (in2_nnz floats) and the mixed operators held in ws (built
 * in FP64 by hx_heff_prepare) -> ws32 (a separate buffer of ws_bytes/2 bytes).
 * Also accepts a prepared VJP plan (hx_heff_vjp_plan_create / hx_heff1_vjp_plan_create),
 * whose coefficient table is then rounded into ws32 as well, for
 * hx_heff_apply_backward_f32. */
int hx_heff_lower_f32(const hx_plan* plan, const double* L, const double* R, const void* ws, float* L32,
                      float* R32, void* ws32, hx_stream stream);

/* sigma32 = H_eff psi32 with FP32 operands and FP32 MFMA accumulation
 * (v_mfma_f32_16x16x4_f32), same blocks and task order as hx_heff_apply.
 * ws32 must hold the result of hx_heff_lower_f32. */
int hx_heff_apply_f32(const hx_plan* plan, const float* L32, const float* R32, void* ws32, const float* psi32,
                      float* sigma32, hx_stream stream);

/* sigma32 = H_eff psi32 with the block products in BF16 on the matrix cores
 * (FP32 accumulation; v_mfma_f32_16x16x32_bf16 on 32-deep K stages with the
 * one-buffer kernel variants 1, 5 and 6, v_mfma_f32_16x16x16_bf16 on 16-deep stages
 * with variants 0 and 4): operands are read in FP32 from the same buffers as
 * hx_heff_apply_f32 and rounded to BF16 (nearest even) when staged, the stage-1
 * intermediate is kept in FP32 between the two rounds.
 * Relative operand precision 2^-9, so sigma carries ~1e-3 relative error; the
 * Davidson work stays FP64 (mixed-precision mode).  Needs a 16-deep kernel
 * variant (HX_EUNSUP for kernel_variant 2). */
int hx_heff_apply_bf16(const hx_plan* plan, const float* L32, const float* R32, void* ws32, const float* psi32,
                       float* sigma32, hx_stream stream);

/* ---- no-allocation sigma-vector ------------------------------------------------ */

/* Size of the library's static device scratch array (per GPU, held until the process
 * ends). */
#define HX_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): sigma = H_eff psi of an uploaded
 * sigma-vector plan from L and R directly -- hx_heff_prepare then hx_heff_apply --
 * with the workspace (mixed operators, intermediates, split-K partials) in a static
 * device array of HX_NOALLOC_SCRATCH_BYTES owned by the library instead of a caller
 * buffer.  Same kernels and summation order as prepare + apply, so sigma is bitwise
 * that of the two calls.  The caller passes L, R, psi and sigma (device, the layouts
 * of hx_heff_apply); sigma is overwritten.  Calls no hipMalloc / hipFree and issues
 * no memset (nothing in the scratch needs clearing).  HX_EINVAL if the plan's
 * ws_bytes exceed HX_NOALLOC_SCRATCH_BYTES, for a plan that is not a sigma-vector
 * plan, a plan not uploaded, or null operands of nonzero length.  All calls on one
 * GPU share that GPU's scratch array: calls that overlap in time on one GPU (other
 * streams, other host threads) race and must be serialised by the caller.  The first
 * call on a device looks up the array's device address (hipGetSymbolAddress) with
 * that device current. */
int hx_heff_apply_noalloc(const hx_plan* plan, const double* L, const double* R, const double* psi,
                          double* sigma, hx_stream stream);

/* ---- Davidson (Davidson 1975; the eigensolver of the sweep) ----------------- */

/* Workspace (bytes) of hx_davidson_step for vectors of length n and basis size <= kmax. */
int64_t hx_davidson_ws_bytes(int64_t n, int32_t kmax);

/* One Davidson step on an orthonormal basis V (k rows of length n, stride ldv)
 * with S = H V (stride lds):
 *   G_ij = v_i . s_j (row/column k-1 computed here; rows < k-1 kept in ws from
 *   earlier calls with the same ws), symmetrised; lowest eigenpair (theta, y) of
 *   G[:k,:k] by Jacobi rotations (largest |y_j| made positive); x = V^T y,
 *   hx = S^T y, r = hx - theta x; t = r / (theta - diag) with |theta - diag|
 *   raised to `guard` (sign kept, + for 0); t orthogonalised against V twice
 *   (classical Gram-Schmidt) and normalised.
 * Outputs (device): x, hx, t (length n) and scal[0] = theta, scal[1] = ||r||,
 * scal[2] = ||t|| before normalisation.  1 <= k <= kmax <= 32.
 * The last 32*32 + 1 doubles of ws keep all eigenvectors of this call's k x k
 * eigensolve (row-major 32 x 32, component i of eigenvector j at [32 i + j]) and
 * then k.  When the next call has k + 1 (the basis grew by one vector), its
 * Jacobi rotations start from those eigenvectors, bordered by a unit vector, and
 * need fewer sweeps; they are used only if orthonormal to 1e-12, so any content
 * of that region gives the same eigenpair up to rounding. */
int hx_davidson_step(int64_t n, int32_t k, int32_t kmax, const double* V, int64_t ldv,
                     const double* S, int64_t lds, const double* diag, double guard, void* ws,
                     double* x, double* hx, double* t, double* scal, hx_stream stream);

/* Thick restart with two vectors: given the current Ritz pair (x, hx = H x, |x| = 1)
 * and the previous iteration's (xp, hxp = H xp), write v1 = the part of xp
 * orthogonal to x (two Gram-Schmidt passes), normalised, and s1 = H v1 by the same
 * linear combination of hx and hxp (no sigma-vector).  scal[3] = |xp - (x.xp) x|
 * before normalisation (0, and v1 = s1 = 0, when xp adds no direction).  The
 * Davidson basis then restarts as [x, v1] instead of [x] alone.  ws: the
 * hx_davidson_step workspace (its projected-matrix rows are not touched). */
int hx_davidson_restart2(int64_t n, const double* x, const double* hx, const double* xp, const double* hxp,
                         double* v1, double* s1, void* ws, double* scal, hx_stream stream);

/* Deterministic FP64 dot products out[j] = a_j . b for j < k (a_j = a + j*lda). */
int hx_dots(int64_t n, int32_t k, const double* a, int64_t lda, const double* b, void* ws,
            double* out, hx_stream stream);

/* x <- x / ||x|| (deterministic FP64 norm; x unchanged if ||x|| = 0); ||x|| -> *norm_out
 * (device).  ws: hx_davidson_ws_bytes(n, 1) bytes of device scratch. */
int hx_normalize(int64_t n, double* x, void* ws, double* norm_out, hx_stream stream);

const char* hx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HEFFX_H */
