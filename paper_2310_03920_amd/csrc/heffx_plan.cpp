// Host-side plan builder: symmetry-sector bookkeeping, MPO operator mixing and
// the owner-computes GEMM task lists of the two-site sigma-vector path and the
// environment updates.  No HIP call is made here, so every function in this file
// runs (and is tested) on a machine without a GPU.
//
// Method (Sec. II.A.1-2, II.C.1): sigma = sum_b Lhat_b psi Rhat_b^T with the
// enlarged-block operators Lhat_b = sum_a L_a (x) W1_ab and Rhat_b = sum_c W2_bc (x) R_c.
// For a fixed middle operator b and a fixed site transition (s' <- s) every
// contributing environment operator has the same quantum-number shift, so the
// sum over a (resp. c) is a plain linear combination of equally shaped
// block-sparse matrices ("mixed operator"; these are the integral-weighted
// complementary-operator sums).  The sigma-vector is then two rounds of block
// GEMMs:  T_b = psi Rhat_b^T  and  sigma += Lhat_b T_b.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "heffx.h"
#include "heffx_internal.h"

namespace hx {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

static const int SITE_Q[4][2] = {{0, 0}, {1, 1}, {1, -1}, {2, 0}};

struct Bond {
    std::vector<std::array<int, 2>> qn;
    std::vector<int> dim;
    // sector lookup: a dense table over the (N, 2Sz) box spanned by the sectors
    int nlo = 0, slo = 0, nw = 0, sw = 0;
    std::vector<int> tab;
    int find(int n, int s) const {
        const int i = n - nlo, j = s - slo;
        if (i < 0 || i >= nw || j < 0 || j >= sw) return -1;
        return tab[(size_t)i * sw + j];
    }
    int nsec() const { return (int)dim.size(); }
};

static bool parse_bond(const hx_bond* b, Bond& out, const char* what) {
    if (!b || b->nsec <= 0 || !b->qn || !b->dim) {
        set_error(std::string(what) + ": empty or null bond table");
        return false;
    }
    out.qn.resize(b->nsec);
    out.dim.resize(b->nsec);
    for (int i = 0; i < b->nsec; ++i) {
        out.qn[i] = {b->qn[2 * i], b->qn[2 * i + 1]};
        out.dim[i] = b->dim[i];
        if (b->dim[i] <= 0) {
            set_error(std::string(what) + ": sector dimension must be positive");
            return false;
        }
        if (i > 0 && !(out.qn[i - 1] < out.qn[i])) {
            set_error(std::string(what) + ": sectors must be strictly increasing in (N, 2Sz)");
            return false;
        }
        if (((out.qn[i][0] - out.qn[i][1]) & 1) != 0) {
            set_error(std::string(what) + ": N and 2Sz must have equal parity");
            return false;
        }
    }
    int nhi = out.qn[0][0], shi = out.qn[0][1];
    out.nlo = nhi;
    out.slo = shi;
    for (const auto& q : out.qn) {
        out.nlo = std::min(out.nlo, q[0]);
        nhi = std::max(nhi, q[0]);
        out.slo = std::min(out.slo, q[1]);
        shi = std::max(shi, q[1]);
    }
    if ((int64_t)(nhi - out.nlo + 1) * (shi - out.slo + 1) > (int64_t)1 << 24) {
        set_error(std::string(what) + ": quantum numbers span too wide a range");
        return false;
    }
    out.nw = nhi - out.nlo + 1;
    out.sw = shi - out.slo + 1;
    out.tab.assign((size_t)out.nw * out.sw, -1);
    for (int i = 0; i < b->nsec; ++i) out.tab[(size_t)(out.qn[i][0] - out.nlo) * out.sw + (out.qn[i][1] - out.slo)] = i;
    return true;
}

struct OpSet {
    std::vector<std::array<int, 2>> dq;
};

static bool parse_ops(const hx_opset* o, OpSet& out, const char* what) {
    if (!o || o->nop < 0 || (o->nop > 0 && !o->dq)) {
        set_error(std::string(what) + ": null operator set");
        return false;
    }
    out.dq.resize(o->nop);
    for (int a = 0; a < o->nop; ++a) out.dq[a] = {o->dq[2 * a], o->dq[2 * a + 1]};
    return true;
}

// Layout of an environment payload (see heffx.h).
struct EnvLayout {
    std::vector<int64_t> op_off;   // nop + 1
    std::vector<int64_t> blk_off;  // nop * nsec, -1 = absent
    int nsec = 0;
    int64_t blk(int a, int isrc) const { return blk_off[(size_t)a * nsec + isrc]; }
};

static EnvLayout env_layout(const Bond& b, const OpSet& ops) {
    EnvLayout L;
    L.nsec = b.nsec();
    int nop = (int)ops.dq.size();
    L.op_off.assign(nop + 1, 0);
    L.blk_off.assign((size_t)nop * L.nsec, -1);
    int64_t o = 0;
    for (int a = 0; a < nop; ++a) {
        L.op_off[a] = o;
        for (int i = 0; i < L.nsec; ++i) {
            int j = b.find(b.qn[i][0] + ops.dq[a][0], b.qn[i][1] + ops.dq[a][1]);
            if (j < 0) continue;
            L.blk_off[(size_t)a * L.nsec + i] = o;
            o += (int64_t)b.dim[j] * b.dim[i];
        }
    }
    L.op_off[nop] = o;
    return L;
}

// Relative block offsets of an operator with shift dq on bond b.
struct ShiftLayout {
    std::vector<int64_t> rel;  // nsec, -1 absent
    int64_t size = 0;
};

static ShiftLayout shift_layout(const Bond& b, int dn, int ds) {
    ShiftLayout s;
    s.rel.assign(b.nsec(), -1);
    for (int i = 0; i < b.nsec(); ++i) {
        int j = b.find(b.qn[i][0] + dn, b.qn[i][1] + ds);
        if (j < 0) continue;
        s.rel[i] = s.size;
        s.size += (int64_t)b.dim[j] * b.dim[i];
    }
    return s;
}

struct PsiBlock {
    int il, s1, s2, ir;
    int64_t off;
};

// Column block of the two-site tensor: all row blocks (il, s1) of the fused
// left sector Q = q(ir) - q(s2), stacked, times the right index of sector ir.
// Stored as one dense (rows x dim(ir)) row-major matrix.
struct PsiCol {
    int s2, ir;
    int rows;                                  // sum of dim(il) over the stacked row blocks
    int64_t off;                               // offset of the column block
    std::vector<std::array<int, 3>> rowblk;    // (il, s1, row offset)
};

struct PsiLayout {
    std::vector<PsiBlock> blocks;
    std::vector<PsiCol> cols;
    std::vector<int> by_key;  // (il, s1, s2) -> block or -1
    int nl = 0;
    int64_t nnz = 0;
    static int64_t key(int il, int s1, int s2) { return ((int64_t)il * 4 + s1) * 4 + s2; }
    int find(int il, int s1, int s2) const {
        if (il < 0 || il >= nl || s1 < 0 || s1 > 3 || s2 < 0 || s2 > 3) return -1;
        return by_key[(size_t)key(il, s1, s2)];
    }
};

// Blocks ordered by column block (s2, ir), then by (il, s1): each column block is a
// contiguous dense matrix and each block a contiguous row range of it.  With
// one_site the second site is absent: s2 = 0 only, with quantum number (0, 0),
// i.e. the one-site tensor (il, s1, ir) grouped by ir.
static PsiLayout psi_layout(const Bond& lb, const Bond& rb, bool one_site = false) {
    PsiLayout P;
    P.nl = lb.nsec();
    P.by_key.assign((size_t)lb.nsec() * 16, -1);
    for (int s2 = 0; s2 < (one_site ? 1 : 4); ++s2)
        for (int ir = 0; ir < rb.nsec(); ++ir) {
            PsiCol c;
            c.s2 = s2;
            c.ir = ir;
            c.rows = 0;
            c.off = P.nnz;
            for (int il = 0; il < lb.nsec(); ++il)
                for (int s1 = 0; s1 < 4; ++s1) {
                    if (lb.qn[il][0] + SITE_Q[s1][0] + SITE_Q[s2][0] != rb.qn[ir][0] ||
                        lb.qn[il][1] + SITE_Q[s1][1] + SITE_Q[s2][1] != rb.qn[ir][1])
                        continue;
                    P.by_key[PsiLayout::key(il, s1, s2)] = (int)P.blocks.size();
                    P.blocks.push_back({il, s1, s2, ir, P.nnz});
                    c.rowblk.push_back({il, s1, c.rows});
                    c.rows += lb.dim[il];
                    P.nnz += (int64_t)lb.dim[il] * rb.dim[ir];
                }
            if (c.rows > 0) P.cols.push_back(std::move(c));
        }
    return P;
}

struct SiteBlock {
    int il, s, ir;
    int64_t off;
};

struct SiteLayout {
    std::vector<SiteBlock> blocks;
    std::vector<int> by_key;  // il*4+s -> block or -1
    int64_t nnz = 0;
    int find(int il, int s) const { return by_key[(size_t)il * 4 + s]; }
};

static SiteLayout site_layout(const Bond& lb, const Bond& rb) {
    SiteLayout S;
    S.by_key.assign((size_t)lb.nsec() * 4, -1);
    for (int il = 0; il < lb.nsec(); ++il)
        for (int s = 0; s < 4; ++s) {
            int ir = rb.find(lb.qn[il][0] + SITE_Q[s][0], lb.qn[il][1] + SITE_Q[s][1]);
            if (ir < 0) continue;
            S.by_key[(size_t)il * 4 + s] = (int)S.blocks.size();
            S.blocks.push_back({il, s, ir, S.nnz});
            S.nnz += (int64_t)lb.dim[il] * rb.dim[ir];
        }
    return S;
}

// ---------------------------------------------------------------- MPO entries

struct Entry {
    int src, tgt;
    double v[16];
};

// Parse MPO entries; `src_is_row` picks which side is the summed environment index.
static bool parse_mpo(const hx_mpo_site* W, const OpSet& rows, const OpSet& cols, bool src_is_row,
                      std::vector<Entry>& out, const char* what) {
    if (!W || W->nnz < 0 || (W->nnz > 0 && (!W->row || !W->col || !W->val))) {
        set_error(std::string(what) + ": null MPO table");
        return false;
    }
    out.clear();
    out.reserve(W->nnz);
    for (int64_t e = 0; e < W->nnz; ++e) {
        int r = W->row[e], c = W->col[e];
        if (r < 0 || r >= (int)rows.dq.size() || c < 0 || c >= (int)cols.dq.size()) {
            set_error(std::string(what) + ": operator index out of range");
            return false;
        }
        int dn = cols.dq[c][0] - rows.dq[r][0], ds = cols.dq[c][1] - rows.dq[r][1];
        Entry en;
        en.src = src_is_row ? r : c;
        en.tgt = src_is_row ? c : r;
        for (int so = 0; so < 4; ++so)
            for (int si = 0; si < 4; ++si) {
                double v = W->val[16 * e + 4 * so + si];
                en.v[4 * so + si] = v;
                if (v != 0.0 && (SITE_Q[so][0] - SITE_Q[si][0] != dn || SITE_Q[so][1] - SITE_Q[si][1] != ds)) {
                    set_error(std::string(what) + ": site matrix breaks (N, 2Sz) conservation");
                    return false;
                }
            }
        out.push_back(en);
    }
    return true;
}

// How a mixed operator (b, s'<-s) is referenced by the GEMM tasks.
struct MixRef {
    int8_t space;    // environment space (alias) or SP_WS (materialised)
    int64_t base;    // element offset of the operator's payload
    int dn, ds;      // shift
    double alpha;
};

struct Trans {
    int so, si;
    MixRef m;
};

struct MixClass {
    int dn, ds;
    std::vector<int> cols;          // source operators with this shift (ascending)
    std::unordered_map<int, int> col_of;
    std::vector<std::vector<std::pair<int, double>>> rows;  // normalised term lists
    int64_t size = 0;               // payload length of one operator
    int64_t ws_base = 0;            // where its rows start in the workspace
};

struct Mixer {
    // input
    const Bond* bond;
    const OpSet* ops;
    const EnvLayout* lay;
    int8_t env_space;
    // output
    std::vector<std::vector<Trans>> trans;  // per target operator
    std::vector<MixClass> classes;
    std::map<std::pair<int, int>, int> class_of;
    double flops = 0;
    int n_mixed = 0;
};

static void build_mixer(Mixer& M, const std::vector<Entry>& ents, int ntgt) {
    M.trans.assign(ntgt, {});
    // terms (tgt, site element t = 4 so + si, src, coef), ordered by (tgt, t, src);
    // the stable sort keeps repeated entries in input order, so their sum is
    // formed in a fixed order
    struct Term {
        int tgt, t, src;
        double v;
    };
    // stable counting sort by target, then a stable sort of each target's terms
    std::vector<int64_t> cnt((size_t)ntgt + 1, 0);
    for (const Entry& e : ents) {
        if ((unsigned)e.tgt >= (unsigned)ntgt) continue;  // parse_mpo keeps targets in range
        for (int t = 0; t < 16; ++t)
            if (e.v[t] != 0.0) ++cnt[(size_t)e.tgt + 1];
    }
    for (int b = 0; b < ntgt; ++b) cnt[(size_t)b + 1] += cnt[(size_t)b];
    std::vector<Term> terms((size_t)cnt[(size_t)ntgt]);
    {
        std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
        for (const Entry& e : ents) {
            if ((unsigned)e.tgt >= (unsigned)ntgt) continue;
            for (int t = 0; t < 16; ++t)
                if (e.v[t] != 0.0) terms[(size_t)pos[(size_t)e.tgt]++] = {e.tgt, t, e.src, e.v[t]};
        }
    }
    for (int b = 0; b < ntgt; ++b)
        std::stable_sort(terms.begin() + cnt[(size_t)b], terms.begin() + cnt[(size_t)b + 1],
                         [](const Term& x, const Term& y) { return x.t != y.t ? x.t < y.t : x.src < y.src; });
    // normalised term list (bytes of (src, coef / first coef) pairs) -> (class, row)
    std::unordered_map<std::string, std::pair<int, int>> seen;
    std::vector<std::pair<int, double>> lst;
    for (size_t g0 = 0; g0 < terms.size();) {
        const int b = terms[g0].tgt, t = terms[g0].t;
        size_t g1 = g0;
        lst.clear();
        while (g1 < terms.size() && terms[g1].tgt == b && terms[g1].t == t) {
            const int src = terms[g1].src;
            double sum = 0.0;
            for (; g1 < terms.size() && terms[g1].tgt == b && terms[g1].t == t && terms[g1].src == src; ++g1)
                sum += terms[g1].v;
            if (sum != 0.0) lst.push_back({src, sum});
        }
        g0 = g1;
        {
            if (lst.empty()) continue;
            const auto& dq = M.ops->dq[lst[0].first];
            Trans tr;
            tr.so = t / 4;
            tr.si = t % 4;
            tr.m.dn = dq[0];
            tr.m.ds = dq[1];
            if (lst.size() == 1) {
                tr.m.space = M.env_space;
                tr.m.base = M.lay->op_off[lst[0].first];
                tr.m.alpha = lst[0].second;
            } else {
                double c0 = lst[0].second;
                std::string key(lst.size() * 12, '\0');
                std::vector<std::pair<int, double>> norm;
                norm.reserve(lst.size());
                for (size_t j = 0; j < lst.size(); ++j) {
                    double v = lst[j].second / c0;
                    std::memcpy(&key[12 * j], &lst[j].first, 4);
                    std::memcpy(&key[12 * j + 4], &v, 8);
                    norm.push_back({lst[j].first, v});
                }
                auto ck = std::make_pair(dq[0], dq[1]);
                int cls;
                auto ci = M.class_of.find(ck);
                if (ci == M.class_of.end()) {
                    cls = (int)M.classes.size();
                    M.class_of[ck] = cls;
                    MixClass mc;
                    mc.dn = dq[0];
                    mc.ds = dq[1];
                    for (int a = 0; a < (int)M.ops->dq.size(); ++a)
                        if (M.ops->dq[a] == dq) {
                            mc.col_of[a] = (int)mc.cols.size();
                            mc.cols.push_back(a);
                        }
                    mc.size = M.lay->op_off[mc.cols[0] + 1] - M.lay->op_off[mc.cols[0]];
                    M.classes.push_back(std::move(mc));
                } else {
                    cls = ci->second;
                }
                auto si = seen.find(key);
                int row;
                if (si != seen.end()) {
                    row = si->second.second;
                } else {
                    row = (int)M.classes[cls].rows.size();
                    M.classes[cls].rows.push_back(norm);
                    seen[key] = {cls, row};
                    M.flops += 2.0 * (double)norm.size() * (double)M.classes[cls].size;
                    M.n_mixed++;
                }
                tr.m.space = SP_WS;
                tr.m.base = -1 - ((int64_t)cls << 32 | row);  // resolved after ws placement
                tr.m.alpha = c0;
            }
            M.trans[b].push_back(tr);
        }
    }
}

// Place materialised mixed operators in the workspace starting at ws0; return end.
static int64_t place_mixer(Mixer& M, int64_t ws0) {
    int64_t o = ws0;
    for (auto& c : M.classes) {
        c.ws_base = o;
        o += c.size * (int64_t)c.rows.size();
    }
    for (auto& tv : M.trans)
        for (auto& tr : tv)
            if (tr.m.space == SP_WS && tr.m.base < 0) {
                int64_t code = -1 - tr.m.base;
                int cls = (int)(code >> 32), row = (int)(code & 0xffffffff);
                tr.m.base = M.classes[cls].ws_base + (int64_t)row * M.classes[cls].size;
            }
    return o;
}

struct Builder {
    Plan* P;
    // Tiles of a block in the order they are dispatched: along the longer side
    // innermost-last, i.e. a wide block column strip by column strip (the row tiles
    // of one strip share its B panel, and the block's few A panels stay cached),
    // a tall block row strip by row strip.
    void add_block_tiles(int shape, int64_t coff, int ldc, int m, int n, int8_t cspace, int8_t beta,
                         int32_t tbeg, int32_t tend, int32_t ktot) {
        const int tm = shape_rows(shape), tn = shape_cols(shape);
        const int nr = (m + tm - 1) / tm, nc = (n + tn - 1) / tn;
        const bool by_col = n > m;
        for (int q = 0; q < nr * nc; ++q) {
            const int r0 = (by_col ? q % nr : q / nc) * tm, c0 = (by_col ? q / nr : q % nc) * tn;
            Tile t;
            t.coff = coff + (int64_t)r0 * ldc + c0;
            t.ldc = ldc;
            t.m = std::min(tm, m - r0);
            t.n = std::min(tn, n - c0);
            t.r0 = r0;
            t.c0 = c0;
            t.tbeg = tbeg;
            t.tend = tend;
            t.ktot = ktot;
            t.set_out(cspace, beta);
            P->tiles.push_back(t);
        }
    }
};

// K of a task as walked by the kernel: padded to the 16-deep LDS stage with zeros.
static inline int32_t kpad(int32_t k, int ks) { return (k + ks - 1) / ks * ks; }

// Kernel variant of a plan (hx_plan_opts.kernel_variant): LDS buffering and K-stage depth.
static int apply_opts(Plan& P, const hx_plan_opts* o) {
    if (o && o->split_kseg_min > 0) P.split_kseg_min = o->split_kseg_min;
    const int v = o ? o->kernel_variant : 0;
    if (v < 0 || v > 6 || v == 3) {
        set_error(v == 3 ? "plan options: kernel_variant 3 (persistent workgroups) was removed"
                         : "plan options: kernel_variant must be 0 .. 6");
        return HX_EINVAL;
    }
    P.variant = v;
    P.kstage = v == 2 ? 8 : 16;
    const int r = (o && o->n_roots > 0) ? o->n_roots : 1;
    if (r > 64) {
        set_error("plan options: n_roots must be at most 64");
        return HX_EINVAL;
    }
    P.n_roots = r;
    const int np = o ? o->b_nparts : 0, pp = o ? o->b_part : 0;
    if (np < 0 || (np > 1 && (pp < 0 || pp >= np)) || (np <= 1 && pp != 0)) {
        set_error("plan options: need 0 <= b_part < b_nparts (or b_nparts <= 1 and b_part = 0)");
        return HX_EINVAL;
    }
    P.b_nparts = np > 1 ? np : 1;
    P.b_part = np > 1 ? pp : 0;
    P.t_merge = !(o && o->t_merge_off != 0);
    return HX_OK;
}

// Split-K: when a launch has too few tiles to fill the GPU, cut long task lists
// at task boundaries into segments that write partial tiles; a reduction then
// sums the partials of each tile in a fixed order (deterministic).
static void split_launch(Plan& P, Launch& L) {
    const int64_t want = 8192;
    if (L.ntile >= want) return;
    int64_t total = 0;
    for (int64_t t = L.tile0; t < L.tile0 + L.ntile; ++t) total += P.tiles[t].ktot;
    const int64_t kseg = std::max<int64_t>(P.split_kseg_min, total / want);
    std::vector<Tile> out;
    int64_t pidx = 0;
    L.red0 = (int64_t)P.reduces.size();
    for (int64_t t = L.tile0; t < L.tile0 + L.ntile; ++t) {
        const Tile tl = P.tiles[t];
        if (tl.ktot <= 2 * kseg) {
            out.push_back(tl);
            continue;
        }
        Reduce r;
        r.coff = tl.coff;
        r.ldc = tl.ldc;
        r.m = tl.m;
        r.n = tl.n;
        r.cspace = (int8_t)tl.cspace();
        r.beta = (int8_t)tl.beta();
        r.pad = 0;
        r.pld = shape_cols(L.shape);
        r.pbase = pidx * TM * TN;
        r.np = 0;
        int32_t a = tl.tbeg;
        while (a < tl.tend) {
            int32_t b = a;
            int64_t ks = 0;
            while (b < tl.tend && (ks < kseg || b == a)) ks += kpad(P.tasks[b++].k, P.kstage);
            Tile p = tl;
            p.tbeg = a;
            p.tend = b;
            p.ktot = (int32_t)ks;
            p.set_out(SP_PART, 0);
            p.coff = pidx * TM * TN;
            p.ldc = shape_cols(L.shape);
            out.push_back(p);
            ++pidx;
            ++r.np;
            a = b;
        }
        P.reduces.push_back(r);
    }
    L.nred = (int64_t)P.reduces.size() - L.red0;
    P.tiles.resize(L.tile0);
    P.tiles.insert(P.tiles.end(), out.begin(), out.end());
    L.ntile = (int64_t)out.size();
    P.part_tiles = std::max(P.part_tiles, pidx);
}

// Order a launch's tiles for the 8 XCDs (workgroup i runs on XCD i mod 8, each XCD
// with its own L2).  Tiles of one output block share their task list and thus
// their operand blocks, so they form a group kept on one XCD, consecutive in its
// dispatch order.  Groups are taken by decreasing work (longest first) and each
// goes to the XCD queue holding the fewest tiles; the queues are then interleaved.
// Indices 0 .. n-1 by decreasing weight (weights >= 0 and finite), ties in
// increasing index.  Large inputs use a stable radix sort on the bit patterns
// (their order is the numeric one for non-negative doubles): the same order as the
// comparison sort, in linear time.
static std::vector<size_t> heaviest_first(const std::vector<double>& w) {
    const size_t n = w.size();
    std::vector<size_t> idx(n);
    std::iota(idx.begin(), idx.end(), (size_t)0);
    if (n < 65536) {
        std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return w[a] > w[b]; });
        return idx;
    }
    std::vector<uint64_t> key(n), kt(n);
    std::vector<size_t> it(n);
    for (size_t i = 0; i < n; ++i) {
        uint64_t b;
        std::memcpy(&b, &w[i], sizeof b);
        key[i] = ~b;  // ascending in ~bits = descending weight
    }
    std::vector<size_t> cnt(65537);
    for (int shift = 0; shift < 64; shift += 16) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (size_t i = 0; i < n; ++i) ++cnt[((key[i] >> shift) & 0xffff) + 1];
        if (cnt[((key[0] >> shift) & 0xffff) + 1] == n) continue;  // one digit value: order kept
        for (size_t d = 1; d < cnt.size(); ++d) cnt[d] += cnt[d - 1];
        for (size_t i = 0; i < n; ++i) {
            const size_t d = cnt[(key[i] >> shift) & 0xffff]++;
            it[d] = idx[i];
            kt[d] = key[i];
        }
        idx.swap(it);
        key.swap(kt);
    }
    return idx;
}

static void sort_tiles(Plan& P, int64_t t0, int64_t n) {
    constexpr int NXCD = 8;
    if (n <= 1) return;
    struct Group {
        int64_t first, count;
        double work;
    };
    std::vector<Group> groups;
    // Non-empty task ranges of one launch are disjoint blocks or split-K segments
    // of them, so distinct groups start at distinct tasks: a group is found by its
    // first task through a direct table (with the range end checked; a hash map
    // takes any range that does not fit that pattern).
    int32_t tlo = INT32_MAX, thi = 0;
    for (int64_t t = 0; t < n; ++t) {
        const Tile& tl = P.tiles[t0 + t];
        if (tl.tbeg != tl.tend) {
            tlo = std::min(tlo, tl.tbeg);
            thi = std::max(thi, tl.tbeg);
        }
    }
    std::vector<int64_t> by_first(tlo <= thi ? (size_t)(thi - tlo + 1) : 0, -1);
    std::unordered_map<uint64_t, size_t> gid;
    std::vector<int32_t> gend;  // range end of each group (non-empty ranges)
    std::vector<size_t> tile_group(n);
    uint64_t prev_key = 0;
    size_t prev_g = SIZE_MAX;
    for (int64_t t = 0; t < n; ++t) {
        const Tile& tl = P.tiles[t0 + t];
        const uint64_t key = ((uint64_t)(uint32_t)tl.tbeg << 32) | (uint32_t)tl.tend;
        size_t g;
        if (tl.tbeg != tl.tend && prev_g != SIZE_MAX && key == prev_key) {
            g = prev_g;  // tiles of one block are mostly emitted one after another
        } else if (tl.tbeg == tl.tend) {  // empty task lists are independent tiles
            g = groups.size();
            groups.push_back({t, 0, 0.0});
            gend.push_back(tl.tend);
        } else {
            int64_t& slot = by_first[(size_t)(tl.tbeg - tlo)];
            if (slot >= 0 && gend[(size_t)slot] == tl.tend) {
                g = (size_t)slot;
            } else {
                auto it = slot >= 0 ? gid.find(key) : gid.end();
                if (it != gid.end()) {
                    g = it->second;
                } else {
                    g = groups.size();
                    groups.push_back({t, 0, 0.0});
                    gend.push_back(tl.tend);
                    if (slot < 0)
                        slot = (int64_t)g;
                    else
                        gid.emplace(key, g);
                }
            }
        }
        prev_key = key;
        prev_g = tl.tbeg != tl.tend ? g : SIZE_MAX;
        tile_group[t] = g;
        groups[g].count++;
        groups[g].work += (double)tl.ktot * tl.m * tl.n;
    }
    // A group of many tiles (a wide block) is cut into runs of at most GMAX
    // consecutive members, so that the XCD queues stay balanced; a run keeps the
    // tiles that share a B panel together (the block's tile order).
    constexpr int64_t GMAX = 32;
    {
        std::vector<int64_t> seen(groups.size(), 0);
        std::vector<size_t> sub(groups.size(), SIZE_MAX);  // current run of each group
        std::vector<Group> runs;
        runs.reserve(groups.size() + (size_t)(n / GMAX));
        for (int64_t t = 0; t < n; ++t) {
            const size_t g = tile_group[t];
            if (seen[g] % GMAX == 0) {
                sub[g] = runs.size();
                runs.push_back({t, 0, 0.0});
            }
            ++seen[g];
            const Tile& tl = P.tiles[t0 + t];
            runs[sub[g]].count++;
            runs[sub[g]].work += (double)tl.ktot * tl.m * tl.n;
            tile_group[t] = sub[g];
        }
        groups.swap(runs);
    }
    // members of each group in increasing tile order (counting sort)
    std::vector<int64_t> mstart(groups.size() + 1, 0), mpos, mlist(n);
    for (int64_t t = 0; t < n; ++t) ++mstart[tile_group[t] + 1];
    for (size_t g = 0; g < groups.size(); ++g) mstart[g + 1] += mstart[g];
    mpos.assign(mstart.begin(), mstart.end() - 1);
    for (int64_t t = 0; t < n; ++t) mlist[mpos[tile_group[t]]++] = t;
    std::vector<double> gw(groups.size());
    for (size_t g = 0; g < gw.size(); ++g) gw[g] = groups[g].work;
    const std::vector<size_t> order = heaviest_first(gw);  // ties in tile order
    std::vector<std::vector<int64_t>> queue(NXCD);
    for (auto& q : queue) q.reserve((size_t)(n / NXCD) + 256);
    for (size_t g : order) {
        int q = 0;
        for (int x = 1; x < NXCD; ++x)
            if (queue[x].size() < queue[q].size()) q = x;
        for (int64_t m = mstart[g]; m < mstart[g + 1]; ++m) queue[q].push_back(mlist[m]);
    }
    std::vector<Tile> out;
    out.reserve(n);
    std::vector<size_t> pos(NXCD, 0);
    for (bool more = true; more;) {
        more = false;
        for (int x = 0; x < NXCD; ++x)
            if (pos[x] < queue[x].size()) {
                out.push_back(P.tiles[t0 + queue[x][pos[x]++]]);
                more = true;
            }
    }
    std::copy(out.begin(), out.end(), P.tiles.begin() + t0);
}

// Emit the mixing GEMMs of a mixer: rows of a class in slabs of TM.
static void emit_mixing(Plan& P, Mixer& M, std::vector<Launch>& seq) {
    if (M.classes.empty()) return;
    Launch L;
    L.kind = NN;
    L.shape = SH_SQ;
    L.stage = P.n_stages++;
    L.tile0 = (int64_t)P.tiles.size();
    L.flops = M.flops;
    Builder B{&P};
    for (auto& c : M.classes) {
        int ncol = (int)c.cols.size();
        int64_t coef0 = (int64_t)P.coef.size();
        P.coef.resize(P.coef.size() + (size_t)ncol * c.rows.size(), 0.0);
        for (size_t r = 0; r < c.rows.size(); ++r)
            for (auto& sc : c.rows[r]) P.coef[coef0 + (int64_t)r * ncol + c.col_of.at(sc.first)] = sc.second;
        int nrow = (int)c.rows.size();
        for (int r0 = 0; r0 < nrow; r0 += TM) {
            int mr = std::min(TM, nrow - r0);
            // columns used by any row of the slab, merged into contiguous runs
            std::vector<char> used(ncol, 0);
            for (int r = r0; r < r0 + mr; ++r)
                for (auto& sc : c.rows[r]) used[c.col_of.at(sc.first)] = 1;
            int32_t tbeg = (int32_t)P.tasks.size();
            int32_t ktot = 0;
            int w = 0;
            while (w < ncol) {
                if (!used[w]) {
                    ++w;
                    continue;
                }
                int w1 = w + 1;
                while (w1 < ncol && used[w1] &&
                       M.lay->op_off[c.cols[w1]] == M.lay->op_off[c.cols[w1 - 1]] + c.size)
                    ++w1;
                Task t;
                t.aoff = coef0 + (int64_t)r0 * ncol + w;
                t.lda = ncol;
                t.boff = M.lay->op_off[c.cols[w]];
                t.ldb = (int32_t)c.size;
                t.k = w1 - w;
                const int ta_ = SP_TAB;
                t.set_spaces(ta_, M.env_space);
                t.alpha = 1.0;
                P.tasks.push_back(t);
                ktot += kpad(t.k, P.kstage);
                w = w1;
            }
            int32_t tend = (int32_t)P.tasks.size();
            // the mixed payload is written in chunks of TN elements; tile n <= TN
            int64_t coff = c.ws_base + (int64_t)r0 * c.size;
            for (int64_t c0 = 0; c0 < c.size; c0 += TN) {
                Tile t;
                t.coff = coff + c0;
                t.ldc = (int32_t)c.size;
                t.m = mr;
                t.n = (int32_t)std::min<int64_t>(TN, c.size - c0);
                t.r0 = 0;
                t.c0 = (int32_t)c0;
                t.tbeg = tbeg;
                t.tend = tend;
                t.ktot = ktot;
                t.set_out(SP_WS, 0);
                P.tiles.push_back(t);
            }
            (void)B;
        }
    }
    L.ntile = (int64_t)P.tiles.size() - L.tile0;
    P.sort_ranges.push_back({L.tile0, L.ntile});  // ordered in finalize_tables
    seq.push_back(L);
}

static int64_t default_budget(const hx_plan_opts* o) {
    int64_t b = (o && o->t_budget_bytes > 0) ? o->t_budget_bytes : ((int64_t)1 << 30);
    return b / 8;  // doubles
}

// ---------------------------------------------------------------- heff plan

struct OutBlockTasks {
    int64_t coff;
    int ldc, m, n;
    std::vector<Task> tasks;
};

// Tile shape of an output block (kernel variants 4 and 5): narrow blocks (at most 32
// columns, more than 64 rows) get 128 x 32 tiles and short ones 32 x 128, so all 4
// waves of a workgroup meet the block; the rest 64 x 64.  Each shape is a launch of
// its own, so a round costs up to three launches (their tails), which the tuner
// weighs against the better-filled workgroups.
// Variant 6: blocks of at most 32 x 32 get single-wave 32 x 32 tiles (no idle waves,
// four times as many tiles in flight per CU), the rest 64 x 64.
static int block_shape(const Plan& P, int m, int n) {
    if (P.variant == 6) return (m <= 32 && n <= 32) ? SH_SMALL : SH_SQ;
    if (P.variant != 4 && P.variant != 5) return SH_SQ;
    if (n <= 32 && m > 64) return SH_TALL;
    if (m <= 32 && n > 64) return SH_WIDE;
    return SH_SQ;
}

// One round of block GEMMs: one launch per tile shape present (their output blocks are
// disjoint, so the launches are independent).
static void flush_blocks(Plan& P, std::vector<OutBlockTasks>& blocks, int kind, int8_t cspace, int8_t beta,
                         bool keep_empty, std::vector<Launch>& seq, double* flops_out, int64_t* ntask_out) {
    const int stage = P.n_stages++;
    for (int sh = SH_SQ; sh <= SH_SMALL; ++sh) {
        Launch L;
        L.kind = kind;
        L.shape = sh;
        L.stage = stage;
        L.tile0 = (int64_t)P.tiles.size();
        L.flops = 0;
        Builder B{&P};
        for (auto& ob : blocks) {
            if (ob.tasks.empty() && !keep_empty) continue;
            if (block_shape(P, ob.m, ob.n) != sh) continue;
            int32_t tbeg = (int32_t)P.tasks.size();
            int32_t ktot = 0;
            for (auto& t : ob.tasks) {
                P.tasks.push_back(t);
                ktot += kpad(t.k, P.kstage);
                L.flops += 2.0 * ob.m * ob.n * (double)t.k;
            }
            int32_t tend = (int32_t)P.tasks.size();
            if (ntask_out) *ntask_out += tend - tbeg;
            B.add_block_tiles(sh, ob.coff, ob.ldc, ob.m, ob.n, cspace, beta, tbeg, tend, ktot);
        }
        L.ntile = (int64_t)P.tiles.size() - L.tile0;
        split_launch(P, L);
        P.sort_ranges.push_back({L.tile0, L.ntile});  // ordered in finalize_tables
        if (flops_out) *flops_out += L.flops;
        if (L.ntile > 0) seq.push_back(L);
    }
}

// The kernels address an operand element relative to its tile's first element
// with a 32-bit offset (at most 128 rows or columns of one block times the leading
// dimension), so leading dimensions are bounded by 2^20.
constexpr int32_t MAX_LD = 1 << 20;

static bool check_task_index_range(const Plan& P) {
    if (P.tasks.size() > (size_t)INT32_MAX) {
        set_error("plan too large: more than 2^31 GEMM tasks");
        return false;
    }
    for (const Task& t : P.tasks)
        if (t.lda > MAX_LD || t.ldb > MAX_LD || t.lda < 0 || t.ldb < 0) {
            set_error("operand leading dimension above 2^20 (block too large)");
            return false;
        }
    return true;
}

// Every copy of the listed gather launches stays inside its source and destination
// buffers (sizes of the plan's operand spaces).
static bool check_gathers(const Plan& P, const std::vector<GatherLaunch>& seq, const char* what) {
    auto space_size = [&](int sp) -> int64_t {
        switch (sp) {
            case SP_L: case SP_GL: return P.in_nnz;
            case SP_R: case SP_GR: return P.in2_nnz;
            case SP_WS: return P.ws_doubles;
            case SP_TAB: return (int64_t)P.coef.size();
            case SP_GW1: return 16 * P.w1_nnz;
            case SP_GW2: return 16 * P.w2_nnz;
            default: return P.psi_nnz;
        }
    };
    for (const GatherLaunch& gl : seq)
        for (int64_t q = gl.g0; q < gl.g0 + gl.ng; ++q) {
            const Gather& g = P.gathers[q];
            const int64_t last = (int64_t)std::max(g.count - 1, 0);
            if (g.count < 0 || g.soff < 0 || g.doff < 0 || g.soff + last * g.sstride >= space_size(g.sspace) ||
                g.doff + last * g.dstride >= space_size(g.dspace)) {
                set_error(std::string("internal: ") + what + " copy out of range");
                return false;
            }
        }
    return true;
}

// one_site: the one-site H_eff (Sec. II.A.2) -- the second site is absent, Mo == Ro and
// e2 is ignored: the right "mixed" operator of middle operator b is R_b itself.
// Hash of an intermediate's psi-side task signature (groups keep first-seen order,
// so the plan does not depend on the hash).
struct SigHash {
    size_t operator()(const std::vector<int64_t>& v) const {
        uint64_t h = 1469598103934665603ull;
        for (int64_t x : v) h = (h ^ (uint64_t)x) * 1099511628211ull;
        return (size_t)(h ^ (h >> 29));
    }
};

static int build_heff(Plan& P, const Bond& lb, const Bond& rb, const OpSet& Lo, const OpSet& Mo,
                      const OpSet& Ro, const std::vector<Entry>& e1, const std::vector<Entry>& e2_in,
                      const hx_plan_opts* opts, bool one_site = false) {
    P.kind = PK_HEFF;
    {
        int rc0 = apply_opts(P, opts);
        if (rc0) return rc0;
    }
    EnvLayout Ll = env_layout(lb, Lo), Rl = env_layout(rb, Ro);
    PsiLayout psi = psi_layout(lb, rb, one_site);
    std::vector<Entry> e2_one;
    if (one_site) {  // identity coupling b -> b on the absent site
        for (int b2 = 0; b2 < (int)Ro.dq.size(); ++b2) {
            Entry en;
            en.src = b2;
            en.tgt = b2;
            for (double& v : en.v) v = 0.0;
            en.v[0] = 1.0;
            e2_one.push_back(en);
        }
    }
    const std::vector<Entry>& e2 = one_site ? e2_one : e2_in;
    // middle-bond part (hx_plan_opts.b_part / b_nparts): only the b dealt to this part
    // get left mixers, so only they become active below
    std::vector<Entry> e1_part;
    const std::vector<Entry>* e1p = &e1;
    if (P.b_nparts > 1) {
        for (const Entry& e : e1)
            if (e.tgt % P.b_nparts == P.b_part) e1_part.push_back(e);
        e1p = &e1_part;
    }
    const int R = P.n_roots;  // roots side by side in every column block (see heffx.h)
    P.psi_nnz = psi.nnz * R;
    P.in_nnz = Ll.op_off.back();
    P.in2_nnz = Rl.op_off.back();

    Mixer ML{&lb, &Lo, &Ll, SP_L, {}, {}, {}, 0, 0};
    Mixer MR{&rb, &Ro, &Rl, SP_R, {}, {}, {}, 0, 0};
    build_mixer(ML, *e1p, (int)Mo.dq.size());
    std::vector<Entry> e2_part;
    if (P.b_nparts > 1) {
        for (const Entry& e : e2)
            if (e.tgt % P.b_nparts == P.b_part) e2_part.push_back(e);
    }
    build_mixer(MR, P.b_nparts > 1 ? e2_part : e2, (int)Mo.dq.size());
    int64_t ws = 0;
    ws = place_mixer(ML, ws);
    ws = place_mixer(MR, ws);
    P.mix_end = ws;
    P.mix_ranges.push_back({0, ws});
    P.n_mixed = ML.n_mixed + MR.n_mixed;
    P.flops_prepare = ML.flops + MR.flops;
    emit_mixing(P, ML, P.prep);
    emit_mixing(P, MR, P.prep);

    // shift layouts of the mixed operators (block offsets relative to the payload)
    std::map<std::pair<int, int>, ShiftLayout> lsh, rsh;
    auto lshift = [&](int dn, int ds) -> const ShiftLayout& {
        auto k = std::make_pair(dn, ds);
        auto it = lsh.find(k);
        if (it == lsh.end()) it = lsh.emplace(k, shift_layout(lb, dn, ds)).first;
        return it->second;
    };
    auto rshift = [&](int dn, int ds) -> const ShiftLayout& {
        auto k = std::make_pair(dn, ds);
        auto it = rsh.find(k);
        if (it == rsh.end()) it = rsh.emplace(k, shift_layout(rb, dn, ds)).first;
        return it->second;
    };

    int nmid = (int)Mo.dq.size();

    // psi column blocks grouped by s2
    std::vector<std::vector<int>> col_by_s2(4);
    for (int c = 0; c < (int)psi.cols.size(); ++c) col_by_s2[psi.cols[c].s2].push_back(c);

    // T sizes per b (for chunking): one stacked column block per (s2', r')
    std::vector<int64_t> tsize(nmid, 0);
    std::vector<char> active(nmid, 0);
    // T blocks of one b are keyed by (s2', r'): a dense index into tables whose
    // entries count as set for b when their stamp is b + 1 (no clearing between b)
    std::vector<int> tstamp((size_t)4 * rb.nsec(), 0), tslot((size_t)4 * rb.nsec(), 0);
    for (int b = 0; b < nmid; ++b) {
        if (ML.trans[b].empty() || MR.trans[b].empty()) continue;
        active[b] = 1;
        for (auto& tr : MR.trans[b])
            for (int ci : col_by_s2[tr.si]) {
                const PsiCol& pc = psi.cols[ci];
                int irp = rb.find(rb.qn[pc.ir][0] + tr.m.dn, rb.qn[pc.ir][1] + tr.m.ds);
                if (irp < 0) continue;
                int& st = tstamp[(size_t)tr.so * rb.nsec() + irp];
                if (st != b + 1) {
                    st = b + 1;
                    tsize[b] += (int64_t)pc.rows * rb.dim[irp] * R;
                }
            }
    }
    std::fill(tstamp.begin(), tstamp.end(), 0);
    int64_t budget = default_budget(opts);
    std::vector<std::pair<int, int>> chunks;  // [b0, b1)
    {
        int b0 = 0;
        int64_t acc = 0;
        for (int b = 0; b < nmid; ++b) {
            if (acc > 0 && acc + tsize[b] > budget) {
                chunks.push_back({b0, b});
                b0 = b;
                acc = 0;
            }
            acc += tsize[b];
        }
        chunks.push_back({b0, nmid});
    }
    int64_t tmax = 0;
    for (auto& ch : chunks) {
        int64_t s = 0;
        for (int b = ch.first; b < ch.second; ++b) s += tsize[b];
        tmax = std::max(tmax, s);
    }
    int64_t t_ws = ws;
    ws += tmax;
    P.n_chunks = (int)chunks.size();

    double fl = 0, useful = 0;
    int64_t nt = 0;
    double tbytes = 0;
    // Rows of a stacked intermediate that stage 2 reads for middle operator b: a row
    // block (l, s1) is read when a left transition of b starts from s1 and maps l into
    // the bond.  Only the span from the first to the last such row is computed (the
    // stacked GEMM stays one operand range); `used` counts the rows read.
    auto read_span = [&](int b, const PsiCol& pc, int& lo, int& hi, int& used) {
        lo = pc.rows;
        hi = 0;
        used = 0;
        for (const auto& rbk : pc.rowblk) {
            const int il = rbk[0], s1 = rbk[1], roff = rbk[2];
            bool read = false;
            for (auto& tr : ML.trans[b])
                if (tr.si == s1 && lb.find(lb.qn[il][0] + tr.m.dn, lb.qn[il][1] + tr.m.ds) >= 0) {
                    read = true;
                    break;
                }
            if (!read) continue;
            lo = std::min(lo, roff);
            hi = std::max(hi, roff + lb.dim[il]);
            used += lb.dim[il];
        }
    };
    // Stacked first-round operands (merged intermediates, below) follow the
    // intermediate region; prepare fills them with gathers after the mixing.
    const bool merge_t = P.t_merge && R == 1;
    const int64_t stack_base = t_ws + tmax;
    int64_t stack_len = 0;
    GatherLaunch stack_gl;
    stack_gl.g0 = (int64_t)P.gathers.size();
    for (size_t ci = 0; ci < chunks.size(); ++ci) {
        // ---- stage 1: T_b[:, (s2', r')] = sum_{s2} psi[:, (s2, r)] Rmix_{b,s2'<-s2}[r', r]^T
        //      on stacked column blocks (all row blocks of one fused sector at once,
        //      restricted to the span of rows that stage 2 reads)
        std::vector<OutBlockTasks> tblocks;
        struct TInfo {
            int b, col, s2p, irp;  // col: the psi column block whose row structure T shares
            int64_t off;
            int rows, r_lo, used;  // stacked rows of the column block; first row held; rows read
            int ld;                // row pitch of the intermediate (wider when merged)
        };
        std::vector<TInfo> tinfo;
        int64_t toff = t_ws;
        for (int b = chunks[ci].first; b < chunks[ci].second; ++b) {
            if (!active[b]) continue;
            for (auto& tr : MR.trans[b]) {
                const ShiftLayout& sl = rshift(tr.m.dn, tr.m.ds);
                for (int cj : col_by_s2[tr.si]) {
                    const PsiCol& pc = psi.cols[cj];
                    int irp = rb.find(rb.qn[pc.ir][0] + tr.m.dn, rb.qn[pc.ir][1] + tr.m.ds);
                    if (irp < 0) continue;
                    const size_t key = (size_t)tr.so * rb.nsec() + irp;
                    int ti;
                    if (tstamp[key] != b + 1) {
                        tstamp[key] = b + 1;
                        int lo, hi, used;
                        read_span(b, pc, lo, hi, used);
                        if (used == 0) {  // nothing of this intermediate is read
                            tslot[key] = -1;
                            continue;
                        }
                        // one T block ((hi - lo) x R*np, roots side by side), one output block per root
                        ti = (int)tinfo.size();
                        tslot[key] = ti;
                        for (int rho = 0; rho < R; ++rho) {
                            OutBlockTasks ob;
                            ob.coff = toff + (int64_t)rho * rb.dim[irp];
                            ob.ldc = R * rb.dim[irp];
                            ob.m = hi - lo;
                            ob.n = rb.dim[irp];
                            tblocks.push_back(std::move(ob));
                        }
                        tinfo.push_back({b, cj, tr.so, irp, toff, pc.rows, lo, used, R * rb.dim[irp]});
                        toff += (int64_t)(hi - lo) * rb.dim[irp] * R;
                    } else {
                        ti = tslot[key];
                        if (ti < 0) continue;
                        if (tinfo[ti].rows != pc.rows) {
                            set_error("internal: stacked intermediate rows inconsistent");
                            return HX_EINVAL;
                        }
                    }
                    const TInfo& tin = tinfo[ti];
                    for (int rho = 0; rho < R; ++rho) {
                        Task t;
                        t.aoff = pc.off * R + (int64_t)tin.r_lo * R * rb.dim[pc.ir] + (int64_t)rho * rb.dim[pc.ir];
                        t.lda = R * rb.dim[pc.ir];
                        t.boff = tr.m.base + sl.rel[pc.ir];
                        t.ldb = rb.dim[pc.ir];
                        t.set_spaces(SP_PSI, tr.m.space);
                        t.k = rb.dim[pc.ir];
                        t.alpha = tr.m.alpha;
                        tblocks[(size_t)ti * R + rho].tasks.push_back(t);
                        useful += 2.0 * tin.used * rb.dim[irp] * (double)t.k;
                    }
                }
            }
        }
        for (auto& ob : tblocks) tbytes += 2.0 * 8.0 * ob.m * ob.n;
        if (merge_t && tinfo.size() > 1) {
            // Intermediates whose task lists agree on the psi side (rows, contraction
            // lengths, order) differ only in the right operator: T_b1 | T_b2 | ... =
            // psi-side product with the stacked operators [a1 Rmix_b1; a2 Rmix_b2; ...].
            // A group becomes one (rows x sum n) matrix; its members are column slices.
            std::unordered_map<std::vector<int64_t>, int, SigHash> gid;
            gid.reserve(tinfo.size());
            std::vector<std::vector<int>> groups;
            for (int ti = 0; ti < (int)tinfo.size(); ++ti) {
                const OutBlockTasks& ob = tblocks[ti];
                std::vector<int64_t> sig;
                sig.reserve(1 + 4 * ob.tasks.size());
                sig.push_back(ob.m);
                for (const Task& t : ob.tasks) {
                    sig.push_back(t.aoff);
                    sig.push_back(t.lda);
                    sig.push_back(t.k);
                    sig.push_back(t.aspace());
                }
                auto ins = gid.emplace(std::move(sig), (int)groups.size());
                if (ins.second) groups.emplace_back();
                groups[(size_t)ins.first->second].push_back(ti);
            }
            std::vector<OutBlockTasks> merged;
            merged.reserve(groups.size());
            int64_t goff = t_ws;
            for (const auto& g : groups) {
                const OutBlockTasks& f = tblocks[(size_t)g[0]];
                int W = 0;
                for (int ti : g) W += tblocks[(size_t)ti].n;
                OutBlockTasks ob;
                ob.coff = goff;
                ob.ldc = W;
                ob.m = f.m;
                ob.n = W;
                int col = 0;
                for (int ti : g) {
                    tinfo[(size_t)ti].off = goff + col;
                    tinfo[(size_t)ti].ld = W;
                    col += tblocks[(size_t)ti].n;
                }
                if (g.size() == 1) {
                    ob.tasks = f.tasks;
                } else {
                    for (size_t j = 0; j < f.tasks.size(); ++j) {
                        Task t = f.tasks[j];
                        const int K = t.k;
                        int64_t row = 0;
                        for (int ti : g) {
                            const Task& u = tblocks[(size_t)ti].tasks[j];
                            const int n = tblocks[(size_t)ti].n;
                            if (u.ldb != K) {
                                set_error("internal: first-round operand block not contiguous");
                                return HX_EINVAL;
                            }
                            Gather gg;
                            gg.soff = u.boff;
                            gg.sspace = (int8_t)u.bspace();
                            gg.sstride = 1;
                            gg.doff = stack_base + stack_len + row * K;
                            gg.dspace = SP_WS;
                            gg.dstride = 1;
                            gg.count = n * K;
                            gg.alpha = u.alpha;
                            gg.pad = 0;
                            P.gathers.push_back(gg);
                            row += n;
                        }
                        t.boff = stack_base + stack_len;
                        t.ldb = K;
                        t.set_spaces(t.aspace(), SP_WS);
                        t.alpha = 1.0;
                        stack_len += (int64_t)W * K;
                        ob.tasks.push_back(t);
                    }
                }
                goff += (int64_t)f.m * W;
                merged.push_back(std::move(ob));
            }
            tblocks.swap(merged);
        }
        flush_blocks(P, tblocks, NT, SP_WS, 0, false, P.apply, &fl, &nt);

        // ---- stage 2: sigma[l',s1',s2',r'] += sum Lmix_{b,s1'<-s1}[l',l] T_b[(l,s1), (s2',r')]
        std::vector<OutBlockTasks> sblocks(psi.blocks.size());
        for (size_t i = 0; i < psi.blocks.size(); ++i) {
            const PsiBlock& pb = psi.blocks[i];
            sblocks[i].coff = pb.off * R;  // all roots of the block: one GEMM with R x the columns
            sblocks[i].ldc = R * rb.dim[pb.ir];
            sblocks[i].m = lb.dim[pb.il];
            sblocks[i].n = R * rb.dim[pb.ir];
        }
        for (const TInfo& ti : tinfo) {
            const PsiCol& pc = psi.cols[ti.col];
            for (const auto& rbk : pc.rowblk) {
                const int il = rbk[0], s1 = rbk[1], roff = rbk[2];
                for (auto& tr : ML.trans[ti.b]) {
                    if (tr.si != s1) continue;
                    int ilp = lb.find(lb.qn[il][0] + tr.m.dn, lb.qn[il][1] + tr.m.ds);
                    if (ilp < 0) continue;
                    int si = psi.find(ilp, tr.so, ti.s2p);
                    if (si < 0 || psi.blocks[si].ir != ti.irp) {
                        set_error("internal: sigma block inconsistent with quantum numbers");
                        return HX_EINVAL;
                    }
                    const ShiftLayout& sl = lshift(tr.m.dn, tr.m.ds);
                    Task t;
                    t.aoff = tr.m.base + sl.rel[il];
                    t.lda = lb.dim[il];
                    const int ta_ = tr.m.space;
                    t.boff = ti.off + (int64_t)(roff - ti.r_lo) * ti.ld;
                    t.ldb = ti.ld;
                    t.set_spaces(ta_, SP_WS);
                    t.k = lb.dim[il];
                    t.alpha = tr.m.alpha;
                    sblocks[si].tasks.push_back(t);
                    useful += 2.0 * sblocks[si].m * (double)sblocks[si].n * t.k;
                }
            }
        }
        flush_blocks(P, sblocks, NN, SP_OUT, ci == 0 ? 0 : 1, ci == 0, P.apply, &fl, &nt);
    }
    P.flops_apply = fl;
    P.flops_useful = useful;
    P.n_tasks_apply = nt;
    for (auto& L : P.apply) P.n_tiles_apply += L.ntile;
    stack_gl.ng = (int64_t)P.gathers.size() - stack_gl.g0;
    if (stack_gl.ng) {
        P.prep_gather.push_back(stack_gl);
        P.mix_ranges.push_back({stack_base, stack_base + stack_len});  // lowered with the mixed operators
        ws = stack_base + stack_len;
    }

    // algorithmic bytes of one apply: psi, sigma, T traffic and every referenced operator once
    {
        double ob = 0;
        std::map<std::pair<int, int64_t>, int64_t> seen;
        for (int b = 0; b < nmid; ++b) {
            if (!active[b]) continue;
            for (auto& tr : ML.trans[b]) seen[{tr.m.space, tr.m.base}] = lshift(tr.m.dn, tr.m.ds).size;
            for (auto& tr : MR.trans[b]) seen[{tr.m.space, tr.m.base}] = rshift(tr.m.dn, tr.m.ds).size;
        }
        for (auto& kv : seen) ob += 8.0 * kv.second;
        P.bytes_apply = ob + 16.0 * psi.nnz * R + tbytes;
    }

    // ---- diagonal: diag[l,s1,s2,r](x,y) = sum_b DL[(l,s1)][x,b] DR[(s2,r)][b,y]
    std::vector<int> b0;
    for (int b = 0; b < nmid; ++b) {
        if (!active[b] || Mo.dq[b][0] != 0 || Mo.dq[b][1] != 0) continue;
        bool l = false, r = false;
        for (auto& tr : ML.trans[b]) l |= (tr.so == tr.si);
        for (auto& tr : MR.trans[b]) r |= (tr.so == tr.si);
        if (l && r) b0.push_back(b);
    }
    int nb0 = (int)b0.size();
    int64_t dl_base = ws;
    std::vector<int64_t> dl_off((size_t)lb.nsec() * 4), dr_off((size_t)rb.nsec() * 4);
    int64_t o = dl_base;
    for (int il = 0; il < lb.nsec(); ++il)
        for (int s = 0; s < 4; ++s) {
            dl_off[(size_t)il * 4 + s] = o;
            o += (int64_t)lb.dim[il] * nb0;
        }
    for (int ir = 0; ir < rb.nsec(); ++ir)
        for (int s = 0; s < 4; ++s) {
            dr_off[(size_t)ir * 4 + s] = o;
            o += (int64_t)rb.dim[ir] * nb0;
        }
    ws = o;
    P.diag_fill.push_back({SP_WS, dl_base, o - dl_base});
    GatherLaunch gl;
    gl.g0 = (int64_t)P.gathers.size();
    for (int j = 0; j < nb0; ++j) {
        int b = b0[j];
        for (auto& tr : ML.trans[b]) {
            if (tr.so != tr.si || tr.m.dn != 0 || tr.m.ds != 0) continue;
            const ShiftLayout& sl = lshift(0, 0);
            for (int il = 0; il < lb.nsec(); ++il) {
                Gather g;
                g.soff = tr.m.base + sl.rel[il];
                g.sstride = lb.dim[il] + 1;
                g.sspace = tr.m.space;
                g.doff = dl_off[(size_t)il * 4 + tr.so] + j;
                g.dstride = nb0;
                g.dspace = SP_WS;
                g.count = lb.dim[il];
                g.alpha = tr.m.alpha;
                g.pad = 0;
                P.gathers.push_back(g);
            }
        }
        for (auto& tr : MR.trans[b]) {
            if (tr.so != tr.si || tr.m.dn != 0 || tr.m.ds != 0) continue;
            const ShiftLayout& sl = rshift(0, 0);
            for (int ir = 0; ir < rb.nsec(); ++ir) {
                Gather g;
                g.soff = tr.m.base + sl.rel[ir];
                g.sstride = rb.dim[ir] + 1;
                g.sspace = tr.m.space;
                g.doff = dr_off[(size_t)ir * 4 + tr.so] + (int64_t)j * rb.dim[ir];
                g.dstride = 1;
                g.dspace = SP_WS;
                g.count = rb.dim[ir];
                g.alpha = tr.m.alpha;
                g.pad = 0;
                P.gathers.push_back(g);
            }
        }
    }
    gl.ng = (int64_t)P.gathers.size() - gl.g0;
    if (gl.ng) P.diag_gather.push_back(gl);
    {
        std::vector<OutBlockTasks> dblocks(psi.blocks.size());
        for (size_t i = 0; i < psi.blocks.size(); ++i) {
            const PsiBlock& pb = psi.blocks[i];
            OutBlockTasks& ob = dblocks[i];
            ob.coff = pb.off;
            ob.ldc = rb.dim[pb.ir];
            ob.m = lb.dim[pb.il];
            ob.n = rb.dim[pb.ir];
            if (nb0 > 0) {
                Task t;
                t.aoff = dl_off[(size_t)pb.il * 4 + pb.s1];
                t.lda = nb0;
                const int ta_ = SP_WS;
                t.boff = dr_off[(size_t)pb.ir * 4 + pb.s2];
                t.ldb = rb.dim[pb.ir];
                t.set_spaces(ta_, SP_WS);
                t.k = nb0;
                t.alpha = 1.0;
                ob.tasks.push_back(t);
            }
        }
        flush_blocks(P, dblocks, NN, SP_OUT, 0, true, P.diag_gemm, nullptr, nullptr);
    }
    P.part_base = ws;
    ws += P.part_tiles * TM * TN;
    P.ws_doubles = ws;
    if (!check_task_index_range(P)) return HX_EINVAL;
    if (!check_gathers(P, P.prep_gather, "stacked operand") || !check_gathers(P, P.diag_gather, "diagonal"))
        return HX_EINVAL;
    return HX_OK;
}


// ---------------------------------------------------------------- adjoint plan
//
// Vector-Jacobian products of sigma = H_eff(L, W1, W2, R) psi with a cotangent g
// (the derivative of a scalar with respect to sigma).  sigma is linear in each
// operand, so with the intermediates of the forward pass,
//   T_b   = psi Rhat_b^T                (recomputed, as in the forward pass)
//   gT_b  = Lhat_b^T g                  (cotangent of T_b)
//   G_t   = g T_b^T   restricted to the (s1' <- s1) rows/cols of transition t = (b, s1', s1)
//   H_t   = gT_b^T psi restricted likewise on the right
//   g_psi = sum_b gT_b Rhat_b
//   g_L_a = sum_t W1_ab[t] G_t,      g_W1_ab[s1', s1] = <L_a, G_(b, s1', s1)>
//   g_R_c = sum_t W2_bc[t] H_t,      g_W2_bc[s2', s2] = <R_c, H_(b, s2', s2)>
// Transitions of one side with equal operator shift form a class: the last two
// lines are then GEMMs with the (transitions x operators) coefficient matrix.

struct GradClass {
    int dn = 0, ds = 0;
    std::vector<int> cols;                       // environment operators with this shift
    std::unordered_map<int, int> col_of;
    std::vector<std::array<int, 3>> trans;       // (b, so, si)
    std::map<std::array<int, 3>, int> t_of;
    std::map<std::pair<int, int>, double> coef;  // (t, col) -> summed site-matrix value
    int64_t size = 0;
    int64_t g_base = 0, gc_base = 0, coef0 = 0;
};

struct GradSide {
    std::vector<GradClass> classes;
    std::map<std::pair<int, int>, int> class_of;
    std::vector<std::vector<std::pair<int, int>>> by_b;  // b -> (class, t)
};

static void build_grad_side(GradSide& G, const std::vector<Entry>& ents, const OpSet& ops, const EnvLayout& lay,
                            int nmid) {
    G.by_b.assign(nmid, {});
    for (const Entry& e : ents)
        for (int t = 0; t < 16; ++t) {
            if (e.v[t] == 0.0) continue;
            const auto& dq = ops.dq[e.src];
            auto ck = std::make_pair(dq[0], dq[1]);
            auto ci = G.class_of.find(ck);
            int c;
            if (ci == G.class_of.end()) {
                c = (int)G.classes.size();
                G.class_of[ck] = c;
                GradClass gc;
                gc.dn = dq[0];
                gc.ds = dq[1];
                for (int a = 0; a < (int)ops.dq.size(); ++a)
                    if (ops.dq[a] == dq) {
                        gc.col_of[a] = (int)gc.cols.size();
                        gc.cols.push_back(a);
                    }
                gc.size = lay.op_off[gc.cols[0] + 1] - lay.op_off[gc.cols[0]];
                G.classes.push_back(std::move(gc));
            } else {
                c = ci->second;
            }
            GradClass& gc = G.classes[c];
            std::array<int, 3> key = {e.tgt, t / 4, t % 4};
            auto ti = gc.t_of.find(key);
            int tix;
            if (ti == gc.t_of.end()) {
                tix = (int)gc.trans.size();
                gc.t_of[key] = tix;
                gc.trans.push_back(key);
                G.by_b[e.tgt].push_back({c, tix});
            } else {
                tix = ti->second;
            }
            gc.coef[{tix, gc.col_of.at(e.src)}] += e.v[t];
        }
}

// Coefficient matrices into the table, transition-gradient and coefficient-gradient
// regions into the workspace.
static int64_t place_grad_side(Plan& P, GradSide& G, int64_t ws) {
    for (auto& gc : G.classes) {
        const int64_t nt = (int64_t)gc.trans.size(), nc = (int64_t)gc.cols.size();
        gc.coef0 = (int64_t)P.coef.size();
        P.coef.resize(P.coef.size() + (size_t)(nt * nc), 0.0);
        for (auto& kv : gc.coef) P.coef[gc.coef0 + kv.first.first * nc + kv.first.second] = kv.second;
        gc.g_base = ws;
        ws += nt * gc.size;
        gc.gc_base = ws;
        ws += nt * nc;
    }
    return ws;
}

// Class GEMMs of one side.  The environment operators of a class are in general not
// adjacent in the payload, so they are staged: copied (before the GEMM launches) into
// a contiguous (operators x payload) matrix for the coefficient gradient
// gC = G_class env^T (NT), and the environment gradient g_env = C^T G_class (TN) is
// written as one contiguous matrix and copied to its operators afterwards.  Each
// class is then one pair of GEMMs with up to 64 operators per tile.
static int64_t grad_class_blocks(Plan& P, const GradSide& G, const EnvLayout& lay, int8_t env_space,
                                 int8_t genv_space, int64_t ws, std::vector<OutBlockTasks>& tn,
                                 std::vector<OutBlockTasks>& nt, std::vector<Gather>& pre,
                                 std::vector<Gather>& post) {
    for (const auto& gc : G.classes) {
        const int ncol = (int)gc.cols.size(), ntr = (int)gc.trans.size();
        if (gc.size <= 0 || ncol == 0) continue;
        const int64_t env_stage = ws, genv_stage = ws + (int64_t)ncol * gc.size;
        ws += 2 * (int64_t)ncol * gc.size;
        for (int w = 0; w < ncol; ++w) {
            Gather g;
            g.soff = lay.op_off[gc.cols[w]];
            g.doff = env_stage + (int64_t)w * gc.size;
            g.sstride = 1;
            g.dstride = 1;
            g.count = (int32_t)gc.size;
            g.sspace = env_space;
            g.dspace = SP_WS;
            g.pad = 0;
            g.alpha = 1.0;
            pre.push_back(g);
            Gather h = g;
            h.soff = genv_stage + (int64_t)w * gc.size;
            h.doff = lay.op_off[gc.cols[w]];
            h.sspace = SP_WS;
            h.dspace = genv_space;
            post.push_back(h);
        }
        // g_env[class] = C^T G_class
        OutBlockTasks ob;
        ob.coff = genv_stage;
        ob.ldc = (int)gc.size;
        ob.m = ncol;
        ob.n = (int)gc.size;
        Task t;
        t.aoff = gc.coef0;
        t.lda = ncol;
        t.boff = gc.g_base;
        t.ldb = (int32_t)gc.size;
        t.k = ntr;
        t.alpha = 1.0;
        t.set_spaces(SP_TAB, SP_WS);
        ob.tasks.push_back(t);
        tn.push_back(std::move(ob));
        // gC = G_class env[class]^T
        OutBlockTasks oc;
        oc.coff = gc.gc_base;
        oc.ldc = ncol;
        oc.m = ntr;
        oc.n = ncol;
        Task u;
        u.aoff = gc.g_base;
        u.lda = (int32_t)gc.size;
        u.boff = env_stage;
        u.ldb = (int32_t)gc.size;
        u.k = (int32_t)gc.size;
        u.alpha = 1.0;
        u.set_spaces(SP_WS, SP_WS);
        oc.tasks.push_back(u);
        nt.push_back(std::move(oc));
    }
    (void)P;
    return ws;
}

// one_site: the adjoint of the one-site sigma-vector (as in build_heff: the second site
// is absent, Mo == Ro, e2 is replaced by the identity coupling b -> b).
static int build_heff_vjp(Plan& P, const Bond& lb, const Bond& rb, const OpSet& Lo, const OpSet& Mo,
                          const OpSet& Ro, const std::vector<Entry>& e1, const std::vector<Entry>& e2_in,
                          const hx_plan_opts* opts, bool one_site = false) {
    P.kind = PK_HEFF_VJP;
    {
        int rc0 = apply_opts(P, opts);
        if (rc0) return rc0;
    }
    if (P.b_nparts != 1) {
        set_error("vjp plan: middle-bond parts (b_nparts > 1) are for sigma-vector plans only");
        return HX_EUNSUP;
    }
    if (P.n_roots != 1) {
        set_error("vjp plan: n_roots must be 1");
        return HX_EUNSUP;
    }
    std::vector<Entry> e2_one;
    if (one_site) {
        for (int b2 = 0; b2 < (int)Ro.dq.size(); ++b2) {
            Entry en;
            en.src = b2;
            en.tgt = b2;
            for (double& v : en.v) v = 0.0;
            en.v[0] = 1.0;
            e2_one.push_back(en);
        }
    }
    const std::vector<Entry>& e2 = one_site ? e2_one : e2_in;
    EnvLayout Ll = env_layout(lb, Lo), Rl = env_layout(rb, Ro);
    PsiLayout psi = psi_layout(lb, rb, one_site);
    P.psi_nnz = psi.nnz;
    P.in_nnz = Ll.op_off.back();
    P.in2_nnz = Rl.op_off.back();
    P.w1_nnz = (int64_t)e1.size();
    P.w2_nnz = (int64_t)e2.size();
    const int nmid = (int)Mo.dq.size();

    // forward mixed operators (hx_heff_prepare on this plan builds them)
    Mixer ML{&lb, &Lo, &Ll, SP_L, {}, {}, {}, 0, 0};
    Mixer MR{&rb, &Ro, &Rl, SP_R, {}, {}, {}, 0, 0};
    build_mixer(ML, e1, nmid);
    build_mixer(MR, e2, nmid);
    int64_t ws = 0;
    ws = place_mixer(ML, ws);
    ws = place_mixer(MR, ws);
    P.mix_end = ws;
    P.mix_ranges.push_back({0, ws});
    P.n_mixed = ML.n_mixed + MR.n_mixed;
    P.flops_prepare = ML.flops + MR.flops;
    emit_mixing(P, ML, P.prep);
    emit_mixing(P, MR, P.prep);

    GradSide GL, GR;
    build_grad_side(GL, e1, Lo, Ll, nmid);
    build_grad_side(GR, e2, Ro, Rl, nmid);
    ws = place_grad_side(P, GL, ws);
    ws = place_grad_side(P, GR, ws);

    std::map<std::pair<int, int>, ShiftLayout> lsh, rsh;
    auto lshift = [&](int dn, int ds) -> const ShiftLayout& {
        auto k = std::make_pair(dn, ds);
        auto it = lsh.find(k);
        if (it == lsh.end()) it = lsh.emplace(k, shift_layout(lb, dn, ds)).first;
        return it->second;
    };
    auto rshift = [&](int dn, int ds) -> const ShiftLayout& {
        auto k = std::make_pair(dn, ds);
        auto it = rsh.find(k);
        if (it == rsh.end()) it = rsh.emplace(k, shift_layout(rb, dn, ds)).first;
        return it->second;
    };

    // wavefunction column block (s2, ir) -> index; row block (il, s1) -> row offset per column
    std::vector<int> col_at((size_t)4 * rb.nsec(), -1);
    std::vector<std::unordered_map<int, int>> roff_of(psi.cols.size());
    for (int c = 0; c < (int)psi.cols.size(); ++c) {
        col_at[(size_t)psi.cols[c].s2 * rb.nsec() + psi.cols[c].ir] = c;
        for (const auto& rbk : psi.cols[c].rowblk) roff_of[c][rbk[0] * 4 + rbk[1]] = rbk[2];
    }
    std::vector<std::vector<int>> col_by_s2(4);
    for (int c = 0; c < (int)psi.cols.size(); ++c) col_by_s2[psi.cols[c].s2].push_back(c);
    // an intermediate column block (T_b or gT_b) is keyed by k = so * nsec + irp; its rows
    // are those of the fused left sector of the wavefunction columns it comes from
    const int nsr = rb.nsec();
    auto target_key = [&](int ir, int so, int dn, int ds) -> int {
        int irp = rb.find(rb.qn[ir][0] + dn, rb.qn[ir][1] + ds);
        return irp < 0 ? -1 : so * nsr + irp;
    };

    // per b: the column blocks of T_b (from the forward right transitions) and of
    // gT_b (also those the right gradient transitions read)
    std::vector<std::vector<int>> tcols(nmid), gtcols(nmid);
    std::vector<std::unordered_map<int, int>> rep(nmid);  // key -> wavefunction column with the same rows
    std::vector<char> need_t(nmid, 0), need_gt(nmid, 0);
    std::vector<int64_t> bsize(nmid, 0);
    for (int b = 0; b < nmid; ++b) {
        need_t[b] = !MR.trans[b].empty() && !GL.by_b[b].empty();
        need_gt[b] = !ML.trans[b].empty() && (!MR.trans[b].empty() || !GR.by_b[b].empty());
        std::vector<char> in_t((size_t)4 * nsr, 0), in_gt((size_t)4 * nsr, 0);
        auto note = [&](int k, int cj) -> bool {
            auto it = rep[b].find(k);
            if (it == rep[b].end()) {
                rep[b][k] = cj;
                return true;
            }
            if (psi.cols[it->second].rows != psi.cols[cj].rows) {
                set_error("internal: stacked intermediate rows inconsistent");
                return false;
            }
            return true;
        };
        for (auto& tr : MR.trans[b])
            for (int cj : col_by_s2[tr.si]) {
                int k = target_key(psi.cols[cj].ir, tr.so, tr.m.dn, tr.m.ds);
                if (k < 0) continue;
                if (!note(k, cj)) return HX_EINVAL;
                in_t[k] = in_gt[k] = 1;
            }
        for (auto& ct : GR.by_b[b]) {
            const GradClass& gc = GR.classes[ct.first];
            const auto& key = gc.trans[ct.second];
            for (int cj : col_by_s2[key[2]]) {
                int k = target_key(psi.cols[cj].ir, key[1], gc.dn, gc.ds);
                if (k < 0) continue;
                if (!note(k, cj)) return HX_EINVAL;
                in_gt[k] = 1;
            }
        }
        for (int k = 0; k < 4 * nsr; ++k) {
            if (!in_t[k] && !in_gt[k]) continue;
            const int64_t sz = (int64_t)psi.cols[rep[b].at(k)].rows * rb.dim[k % nsr];
            if (need_t[b] && in_t[k]) {
                tcols[b].push_back(k);
                bsize[b] += sz;
            }
            if (need_gt[b] && in_gt[k]) {
                gtcols[b].push_back(k);
                bsize[b] += sz;
            }
        }
    }
    const int64_t budget = default_budget(opts);
    std::vector<std::pair<int, int>> chunks;
    {
        int b0 = 0;
        int64_t acc = 0;
        for (int b = 0; b < nmid; ++b) {
            if (acc > 0 && acc + bsize[b] > budget) {
                chunks.push_back({b0, b});
                b0 = b;
                acc = 0;
            }
            acc += bsize[b];
        }
        chunks.push_back({b0, nmid});
    }
    int64_t cmax = 0;
    for (auto& ch : chunks) {
        int64_t sz = 0;
        for (int b = ch.first; b < ch.second; ++b) sz += bsize[b];
        cmax = std::max(cmax, sz);
    }
    const int64_t t_ws = ws;
    ws += cmax;
    P.n_chunks = (int)chunks.size();

    P.bw_fill.push_back({SP_GL, 0, P.in_nnz});
    P.bw_fill.push_back({SP_GR, 0, P.in2_nnz});
    P.bw_fill.push_back({SP_GW1, 0, 16 * P.w1_nnz});
    P.bw_fill.push_back({SP_GW2, 0, 16 * P.w2_nnz});

    double fl = 0;
    int64_t ntask = 0;
    std::vector<int64_t> toff(psi.cols.size()), gtoff(psi.cols.size());
    for (size_t ci = 0; ci < chunks.size(); ++ci) {
        // intermediates of the chunk: T_b then gT_b column blocks per b
        std::vector<std::unordered_map<int, int64_t>> T(nmid), GT(nmid);
        int64_t o = t_ws;
        for (int b = chunks[ci].first; b < chunks[ci].second; ++b) {
            for (int k : tcols[b]) {
                T[b][k] = o;
                o += (int64_t)psi.cols[rep[b].at(k)].rows * rb.dim[k % nsr];
            }
            for (int k : gtcols[b]) {
                GT[b][k] = o;
                o += (int64_t)psi.cols[rep[b].at(k)].rows * rb.dim[k % nsr];
            }
        }
        // ---- T_b = psi Rhat_b^T (NT), as in the forward pass
        {
            std::vector<OutBlockTasks> blocks;
            for (int b = chunks[ci].first; b < chunks[ci].second; ++b) {
                if (!need_t[b]) continue;
                std::unordered_map<int, int> bi;
                for (int k : tcols[b]) {
                    bi[k] = (int)blocks.size();
                    OutBlockTasks ob;
                    ob.coff = T[b][k];
                    ob.ldc = rb.dim[k % nsr];
                    ob.m = psi.cols[rep[b].at(k)].rows;
                    ob.n = rb.dim[k % nsr];
                    blocks.push_back(std::move(ob));
                }
                for (auto& tr : MR.trans[b]) {
                    const ShiftLayout& sl = rshift(tr.m.dn, tr.m.ds);
                    for (int cj : col_by_s2[tr.si]) {
                        const PsiCol& pc = psi.cols[cj];
                        int c = target_key(pc.ir, tr.so, tr.m.dn, tr.m.ds);
                        if (c < 0) continue;
                        Task t;
                        t.aoff = pc.off;
                        t.lda = rb.dim[pc.ir];
                        t.boff = tr.m.base + sl.rel[pc.ir];
                        t.ldb = rb.dim[pc.ir];
                        t.k = rb.dim[pc.ir];
                        t.alpha = tr.m.alpha;
                        t.set_spaces(SP_PSI, tr.m.space);
                        blocks[bi.at(c)].tasks.push_back(t);
                    }
                }
            }
            flush_blocks(P, blocks, NT, SP_WS, 0, true, P.apply, &fl, &ntask);
        }
        // ---- gT_b = Lhat_b^T g (TN), one output block per (column, row block)
        {
            std::vector<OutBlockTasks> blocks;
            for (int b = chunks[ci].first; b < chunks[ci].second; ++b) {
                if (!need_gt[b]) continue;
                for (int c : gtcols[b]) {
                    const PsiCol& pc = psi.cols[rep[b].at(c)];
                    const int n = rb.dim[c % nsr], s2p = c / nsr, irp = c % nsr;
                    for (const auto& rbk : pc.rowblk) {
                        const int il = rbk[0], s1 = rbk[1];
                        OutBlockTasks ob;
                        ob.coff = GT[b][c] + (int64_t)rbk[2] * n;
                        ob.ldc = n;
                        ob.m = lb.dim[il];
                        ob.n = n;
                        for (auto& tr : ML.trans[b]) {
                            if (tr.si != s1) continue;
                            int ilp = lb.find(lb.qn[il][0] + tr.m.dn, lb.qn[il][1] + tr.m.ds);
                            if (ilp < 0) continue;
                            int gi = psi.find(ilp, tr.so, s2p);
                            if (gi < 0 || psi.blocks[gi].ir != irp) {
                                set_error("internal: cotangent block inconsistent with quantum numbers");
                                return HX_EINVAL;
                            }
                            const ShiftLayout& sl = lshift(tr.m.dn, tr.m.ds);
                            Task t;
                            t.aoff = tr.m.base + sl.rel[il];
                            t.lda = lb.dim[il];
                            t.boff = psi.blocks[gi].off;
                            t.ldb = n;
                            t.k = lb.dim[ilp];
                            t.alpha = tr.m.alpha;
                            t.set_spaces(tr.m.space, SP_G);
                            ob.tasks.push_back(t);
                        }
                        blocks.push_back(std::move(ob));
                    }
                }
            }
            flush_blocks(P, blocks, TN_, SP_WS, 0, true, P.apply, &fl, &ntask);
        }
        // ---- G_t = g T_b^T on the rows/cols of t (NT)
        {
            std::vector<OutBlockTasks> blocks;
            for (int b = chunks[ci].first; b < chunks[ci].second; ++b) {
                // output blocks (t, il) of this b (zero when T_b vanishes)
                std::map<std::pair<int, int>, int> out_of;  // ((class<<20)|t, il) -> block
                for (auto& ct : GL.by_b[b]) {
                    const GradClass& gc = GL.classes[ct.first];
                    const ShiftLayout& sl = lshift(gc.dn, gc.ds);
                    for (int il = 0; il < lb.nsec(); ++il) {
                        if (sl.rel[il] < 0) continue;
                        int ilp = lb.find(lb.qn[il][0] + gc.dn, lb.qn[il][1] + gc.ds);
                        OutBlockTasks ob;
                        ob.coff = gc.g_base + (int64_t)ct.second * gc.size + sl.rel[il];
                        ob.ldc = lb.dim[il];
                        ob.m = lb.dim[ilp];
                        ob.n = lb.dim[il];
                        out_of[{(ct.first << 20) | ct.second, il}] = (int)blocks.size();
                        blocks.push_back(std::move(ob));
                    }
                }
                if (!need_t[b]) continue;
                for (int c : tcols[b]) {
                    const PsiCol& pc = psi.cols[rep[b].at(c)];
                    const int n = rb.dim[c % nsr], s2p = c / nsr, irp = c % nsr;
                    for (const auto& rbk : pc.rowblk) {
                        const int il = rbk[0], s1 = rbk[1];
                        for (auto& ct : GL.by_b[b]) {
                            const GradClass& gc = GL.classes[ct.first];
                            const auto& key = gc.trans[ct.second];
                            if (key[2] != s1) continue;
                            int ilp = lb.find(lb.qn[il][0] + gc.dn, lb.qn[il][1] + gc.ds);
                            if (ilp < 0) continue;
                            int gi = psi.find(ilp, key[1], s2p);
                            if (gi < 0 || psi.blocks[gi].ir != irp) continue;
                            Task t;
                            t.aoff = psi.blocks[gi].off;
                            t.lda = n;
                            t.boff = T[b][c] + (int64_t)rbk[2] * n;
                            t.ldb = n;
                            t.k = n;
                            t.alpha = 1.0;
                            t.set_spaces(SP_G, SP_WS);
                            blocks[out_of.at({(ct.first << 20) | ct.second, il})].tasks.push_back(t);
                        }
                    }
                }
            }
            flush_blocks(P, blocks, NT, SP_WS, 0, true, P.apply, &fl, &ntask);
        }
        // ---- g_psi += gT_b Rhat_b (NN), summed over the chunk's b
        {
            std::vector<OutBlockTasks> blocks(psi.cols.size());
            for (size_t c = 0; c < psi.cols.size(); ++c) {
                blocks[c].coff = psi.cols[c].off;
                blocks[c].ldc = rb.dim[psi.cols[c].ir];
                blocks[c].m = psi.cols[c].rows;
                blocks[c].n = rb.dim[psi.cols[c].ir];
            }
            for (int b = chunks[ci].first; b < chunks[ci].second; ++b) {
                if (!need_gt[b]) continue;
                for (auto& tr : MR.trans[b]) {
                    const ShiftLayout& sl = rshift(tr.m.dn, tr.m.ds);
                    for (int cj : col_by_s2[tr.si]) {
                        const PsiCol& pc = psi.cols[cj];
                        int c = target_key(pc.ir, tr.so, tr.m.dn, tr.m.ds);
                        if (c < 0) continue;
                        const int np = rb.dim[c % nsr];
                        Task t;
                        t.aoff = GT[b].at(c);
                        t.lda = np;
                        t.boff = tr.m.base + sl.rel[pc.ir];
                        t.ldb = rb.dim[pc.ir];
                        t.k = np;
                        t.alpha = tr.m.alpha;
                        t.set_spaces(SP_WS, tr.m.space);
                        blocks[cj].tasks.push_back(t);
                    }
                }
            }
            flush_blocks(P, blocks, NN, SP_OUT, ci == 0 ? 0 : 1, ci == 0, P.apply, &fl, &ntask);
        }
        // ---- H_t = gT_b^T psi on the rows/cols of t (TN)
        {
            std::vector<OutBlockTasks> blocks;
            for (int b = chunks[ci].first; b < chunks[ci].second; ++b) {
                for (auto& ct : GR.by_b[b]) {
                    const GradClass& gc = GR.classes[ct.first];
                    const auto& key = gc.trans[ct.second];
                    const ShiftLayout& sl = rshift(gc.dn, gc.ds);
                    for (int ir = 0; ir < rb.nsec(); ++ir) {
                        if (sl.rel[ir] < 0) continue;
                        int irp = rb.find(rb.qn[ir][0] + gc.dn, rb.qn[ir][1] + gc.ds);
                        OutBlockTasks ob;
                        ob.coff = gc.g_base + (int64_t)ct.second * gc.size + sl.rel[ir];
                        ob.ldc = rb.dim[ir];
                        ob.m = rb.dim[irp];
                        ob.n = rb.dim[ir];
                        int cj = col_at[(size_t)key[2] * rb.nsec() + ir];
                        int c = key[1] * nsr + irp;
                        if (need_gt[b] && cj >= 0 && c >= 0) {
                            auto it = GT[b].find(c);
                            if (it == GT[b].end()) {
                                set_error("internal: missing cotangent intermediate");
                                return HX_EINVAL;
                            }
                            Task t;
                            t.aoff = it->second;
                            t.lda = rb.dim[irp];
                            t.boff = psi.cols[cj].off;
                            t.ldb = rb.dim[ir];
                            t.k = psi.cols[cj].rows;
                            t.alpha = 1.0;
                            t.set_spaces(SP_WS, SP_PSI);
                            ob.tasks.push_back(t);
                        }
                        blocks.push_back(std::move(ob));
                    }
                }
            }
            flush_blocks(P, blocks, TN_, SP_WS, 0, true, P.apply, &fl, &ntask);
        }
    }
    // ---- class GEMMs: environment gradients (TN) and coefficient gradients (NT),
    // on class-contiguous staged copies
    {
        std::vector<OutBlockTasks> tn, nt;
        std::vector<Gather> pre, post;
        ws = grad_class_blocks(P, GL, Ll, SP_L, SP_GL, ws, tn, nt, pre, post);
        ws = grad_class_blocks(P, GR, Rl, SP_R, SP_GR, ws, tn, nt, pre, post);
        flush_blocks(P, tn, TN_, SP_WS, 0, false, P.apply, &fl, &ntask);
        flush_blocks(P, nt, NT, SP_WS, 0, false, P.apply, &fl, &ntask);
        if (!pre.empty()) {
            P.bw_pre.push_back({(int64_t)P.gathers.size(), (int64_t)pre.size()});
            P.gathers.insert(P.gathers.end(), pre.begin(), pre.end());
        }
        if (!post.empty()) {
            P.bw_post.push_back({(int64_t)P.gathers.size(), (int64_t)post.size()});
            P.gathers.insert(P.gathers.end(), post.begin(), post.end());
        }
    }
    // ---- scatter the coefficient gradients to the MPO value layout
    {
        GatherLaunch gl;
        gl.g0 = (int64_t)P.gathers.size();
        auto emit = [&](const GradSide& G, const std::vector<Entry>& ents, const OpSet& ops, int8_t dspace) {
            for (size_t e = 0; e < ents.size(); ++e) {
                const Entry& en = ents[e];
                const auto& dq = ops.dq[en.src];
                const GradClass& gc = G.classes[G.class_of.at({dq[0], dq[1]})];
                for (int t = 0; t < 16; ++t) {
                    if (en.v[t] == 0.0) continue;
                    int tix = gc.t_of.at({en.tgt, t / 4, t % 4});
                    Gather g;
                    g.soff = gc.gc_base + (int64_t)tix * (int64_t)gc.cols.size() + gc.col_of.at(en.src);
                    g.doff = (int64_t)e * 16 + t;
                    g.sstride = 1;
                    g.dstride = 1;
                    g.count = 1;
                    g.sspace = SP_WS;
                    g.dspace = dspace;
                    g.pad = 0;
                    g.alpha = 1.0;
                    P.gathers.push_back(g);
                }
            }
        };
        emit(GL, e1, Lo, SP_GW1);
        emit(GR, e2, Ro, SP_GW2);
        gl.ng = (int64_t)P.gathers.size() - gl.g0;
        if (gl.ng) P.bw_gather.push_back(gl);
    }
    P.flops_apply = fl;
    P.n_tasks_apply = ntask;
    for (auto& L : P.apply) P.n_tiles_apply += L.ntile;
    P.coef32_base = ws;  // FP32 coefficient table of the FP32 backward (hx_heff_lower_f32)
    ws += (int64_t)P.coef.size();
    P.part_base = ws;
    ws += P.part_tiles * TM * TN;
    P.ws_doubles = ws;
    if (!check_task_index_range(P)) return HX_EINVAL;
    // every copy of the adjoint stays inside its source and destination buffers
    auto space_size = [&](int sp) -> int64_t {
        switch (sp) {
            case SP_L: case SP_GL: return P.in_nnz;
            case SP_R: case SP_GR: return P.in2_nnz;
            case SP_WS: return P.ws_doubles;
            case SP_TAB: return (int64_t)P.coef.size();
            case SP_GW1: return 16 * P.w1_nnz;
            case SP_GW2: return 16 * P.w2_nnz;
            default: return P.psi_nnz;
        }
    };
    for (auto* seq : {&P.bw_pre, &P.bw_post, &P.bw_gather})
        for (const GatherLaunch& gl : *seq)
            for (int64_t q = gl.g0; q < gl.g0 + gl.ng; ++q) {
                const Gather& g = P.gathers[q];
                const int64_t last = (int64_t)std::max(g.count - 1, 0);
                if (g.count < 0 || g.soff < 0 || g.doff < 0 ||
                    g.soff + last * g.sstride >= space_size(g.sspace) ||
                    g.doff + last * g.dstride >= space_size(g.dspace)) {
                    set_error("internal: adjoint copy out of range");
                    return HX_EINVAL;
                }
            }
    return HX_OK;
}

// ---------------------------------------------------------------- env plans

static int build_env(Plan& P, int dir, const Bond& bin, const Bond& bout, const OpSet& oin, const OpSet& oout,
                     const std::vector<Entry>& ents, const hx_plan_opts* opts) {
    // dir 0: bin = bond k (lb), bout = bond k+1; site tensor between bin and bout.
    // dir 1: bin = bond k+1 (rb), bout = bond k; site tensor between bout and bin.
    P.kind = dir == 0 ? PK_ENV_LEFT : PK_ENV_RIGHT;
    {
        int rc0 = apply_opts(P, opts);
        if (rc0) return rc0;
    }
    if (P.b_nparts != 1) {
        set_error("env plan: middle-bond parts (b_nparts > 1) are for sigma-vector plans only");
        return HX_EUNSUP;
    }
    EnvLayout Lin = env_layout(bin, oin), Lout = env_layout(bout, oout);
    SiteLayout S = dir == 0 ? site_layout(bin, bout) : site_layout(bout, bin);
    P.in_nnz = Lin.op_off.back();
    P.in2_nnz = S.nnz;
    P.out_nnz = Lout.op_off.back();
    Mixer M{&bin, &oin, &Lin, SP_PSI, {}, {}, {}, 0, 0};
    build_mixer(M, ents, (int)oout.dq.size());
    int64_t ws = place_mixer(M, 0);
    P.n_mixed = M.n_mixed;
    P.flops_prepare = M.flops;
    emit_mixing(P, M, P.apply);  // env update = mixing + E1 + E2 in one call

    std::map<std::pair<int, int>, ShiftLayout> shl;
    auto shift = [&](int dn, int ds) -> const ShiftLayout& {
        auto k = std::make_pair(dn, ds);
        auto it = shl.find(k);
        if (it == shl.end()) it = shl.emplace(k, shift_layout(bin, dn, ds)).first;
        return it->second;
    };
    int nout = (int)oout.dq.size();
    // site blocks grouped by site state
    std::vector<std::vector<int>> by_s(4);
    for (int i = 0; i < (int)S.blocks.size(); ++i) by_s[S.blocks[i].s].push_back(i);

    // intermediate blocks are keyed by (xp, so, y): a dense index; per operator b a
    // table entry counts as set when its stamp is b + 1 (no clearing between b)
    const int64_t nkey = (int64_t)bin.nsec() * 4 * bout.nsec();
    auto ykey = [&](int xp, int so, int y) { return ((int64_t)xp * 4 + so) * bout.nsec() + y; };
    std::vector<int> stamp((size_t)nkey, 0), slot((size_t)nkey, 0);
    // intermediate size per b
    std::vector<int64_t> ysize(nout, 0);
    for (int b = 0; b < nout; ++b) {
        for (auto& tr : M.trans[b])
            for (int si : by_s[tr.si]) {
                const SiteBlock& sb = S.blocks[si];
                int x = dir == 0 ? sb.il : sb.ir;   // the index the mixed op acts on (in bin)
                int xp = bin.find(bin.qn[x][0] + tr.m.dn, bin.qn[x][1] + tr.m.ds);
                if (xp < 0) continue;
                int y = dir == 0 ? sb.ir : sb.il;   // the free index (in bout)
                int& st = stamp[(size_t)ykey(xp, tr.so, y)];
                if (st != b + 1) {
                    st = b + 1;
                    ysize[b] += (int64_t)bin.dim[xp] * bout.dim[y];
                }
            }
    }
    std::fill(stamp.begin(), stamp.end(), 0);
    int64_t budget = default_budget(opts);
    std::vector<std::pair<int, int>> chunks;
    {
        int b0 = 0;
        int64_t acc = 0;
        for (int b = 0; b < nout; ++b) {
            if (acc > 0 && acc + ysize[b] > budget) {
                chunks.push_back({b0, b});
                b0 = b;
                acc = 0;
            }
            acc += ysize[b];
        }
        chunks.push_back({b0, nout});
    }
    int64_t ymax = 0;
    for (auto& ch : chunks) {
        int64_t s = 0;
        for (int b = ch.first; b < ch.second; ++b) s += ysize[b];
        ymax = std::max(ymax, s);
    }
    int64_t y_ws = ws;
    ws += ymax;
    P.n_chunks = (int)chunks.size();
    double fl = 0;
    int64_t nt = 0;
    for (auto& ch : chunks) {
        std::vector<OutBlockTasks> yblocks;
        struct YInfo {
            int b, xp, so, y;
            int64_t off;
        };
        std::vector<YInfo> yinfo;
        int64_t yoff = y_ws;
        for (int b = ch.first; b < ch.second; ++b) {
            for (auto& tr : M.trans[b]) {
                const ShiftLayout& sl = shift(tr.m.dn, tr.m.ds);
                for (int si : by_s[tr.si]) {
                    const SiteBlock& sb = S.blocks[si];
                    int x = dir == 0 ? sb.il : sb.ir;
                    int y = dir == 0 ? sb.ir : sb.il;
                    int xp = bin.find(bin.qn[x][0] + tr.m.dn, bin.qn[x][1] + tr.m.ds);
                    if (xp < 0) continue;
                    const size_t key = (size_t)ykey(xp, tr.so, y);
                    int yi;
                    if (stamp[key] != b + 1) {
                        yi = (int)yblocks.size();
                        stamp[key] = b + 1;
                        slot[key] = yi;
                        OutBlockTasks ob;
                        ob.coff = yoff;
                        ob.m = bin.dim[xp];
                        ob.n = bout.dim[y];
                        ob.ldc = ob.n;
                        yblocks.push_back(std::move(ob));
                        yinfo.push_back({b, xp, tr.so, y, yoff});
                        yoff += (int64_t)bin.dim[xp] * bout.dim[y];
                    } else {
                        yi = slot[key];
                    }
                    Task t;
                    t.aoff = tr.m.base + sl.rel[x];   // mixed op block (xp <- x)
                    t.lda = bin.dim[x];
                    const int ta_ = tr.m.space;
                    t.boff = sb.off;                  // site block
                    t.ldb = dir == 0 ? bout.dim[y] : bin.dim[x];
                    t.set_spaces(ta_, SP_R);
                    t.k = bin.dim[x];
                        t.alpha = tr.m.alpha;
                    yblocks[yi].tasks.push_back(t);
                }
            }
        }
        flush_blocks(P, yblocks, dir == 0 ? NN : NT, SP_WS, 0, false, P.apply, &fl, &nt);

        // E2: out_b[y' <- y] = sum_{(xp, so)} op(site[(xp,so) -> y']) Y_b[xp, so, y]
        std::vector<OutBlockTasks> oblocks;
        // output block of (b, y) in this chunk, or -1
        std::vector<int> oidx((size_t)(ch.second - ch.first) * bout.nsec(), -1);
        for (int b = ch.first; b < ch.second; ++b)
            for (int y = 0; y < bout.nsec(); ++y) {
                int64_t off = Lout.blk(b, y);
                if (off < 0) continue;
                int yp = bout.find(bout.qn[y][0] + oout.dq[b][0], bout.qn[y][1] + oout.dq[b][1]);
                OutBlockTasks ob;
                ob.coff = off;
                ob.m = bout.dim[yp];
                ob.n = bout.dim[y];
                ob.ldc = ob.n;
                oidx[(size_t)(b - ch.first) * bout.nsec() + y] = (int)oblocks.size();
                oblocks.push_back(std::move(ob));
            }
        for (const YInfo& yi : yinfo) {
            int yp = bout.find(bout.qn[yi.y][0] + oout.dq[yi.b][0], bout.qn[yi.y][1] + oout.dq[yi.b][1]);
            if (yp < 0) continue;
            int sbk;
            if (dir == 0) {
                sbk = S.find(yi.xp, yi.so);  // A block (xp, so) -> must land on yp
                if (sbk < 0 || S.blocks[sbk].ir != yp) continue;
            } else {
                sbk = S.find(yp, yi.so);     // B block (yp, so) -> must land on xp
                if (sbk < 0 || S.blocks[sbk].ir != yi.xp) continue;
            }
            const int ob_i = oidx[(size_t)(yi.b - ch.first) * bout.nsec() + yi.y];
            if (ob_i < 0) {
                set_error("internal: environment block missing");
                return HX_EINVAL;
            }
            Task t;
            t.aoff = S.blocks[sbk].off;
            t.lda = dir == 0 ? bout.dim[yp] : bin.dim[yi.xp];
            const int ta_ = SP_R;
            t.boff = yi.off;
            t.ldb = bout.dim[yi.y];
            t.set_spaces(ta_, SP_WS);
            t.k = bin.dim[yi.xp];
            t.alpha = 1.0;
            oblocks[ob_i].tasks.push_back(t);
        }
        flush_blocks(P, oblocks, dir == 0 ? TN_ : NN, SP_OUT, 0, true, P.apply, &fl, &nt);
    }
    P.flops_apply = fl + M.flops;
    P.n_tasks_apply = nt;
    for (auto& L : P.apply) P.n_tiles_apply += L.ntile;
    P.part_base = ws;
    ws += P.part_tiles * TM * TN;
    P.ws_doubles = ws;
    P.bytes_apply = 8.0 * (P.in_nnz + P.in2_nnz + P.out_nnz);
    if (!check_task_index_range(P)) return HX_EINVAL;
    return HX_OK;
}

// Every element a GEMM launch of the plan can touch lies inside its operand space:
// for each tile, the output rows and columns of its extent, and for each of its
// tasks the A rows x k and k x B columns that the kernel loads (its loads stay
// inside the tile's extent and the task's k).  Split-K partial tiles and their
// reductions stay inside the partial region.  Checked once per plan on the host.
static int check_gemm_bounds(const Plan& P) {
    const bool env = P.kind == PK_ENV_LEFT || P.kind == PK_ENV_RIGHT;
    int64_t size[SP_N];
    size[SP_PSI] = env ? P.in_nnz : P.psi_nnz;
    size[SP_OUT] = env ? P.out_nnz : P.psi_nnz;
    size[SP_L] = env ? 0 : P.in_nnz;
    size[SP_R] = P.in2_nnz;
    size[SP_WS] = P.ws_doubles;
    size[SP_TAB] = (int64_t)P.coef.size();
    size[SP_PART] = P.ws_doubles - P.part_base;
    size[SP_G] = P.kind == PK_HEFF_VJP ? P.psi_nnz : 0;
    size[SP_GL] = P.kind == PK_HEFF_VJP ? P.in_nnz : 0;
    size[SP_GR] = P.kind == PK_HEFF_VJP ? P.in2_nnz : 0;
    size[SP_GW1] = P.kind == PK_HEFF_VJP ? 16 * P.w1_nnz : 0;
    size[SP_GW2] = P.kind == PK_HEFF_VJP ? 16 * P.w2_nnz : 0;
    auto inside = [&](int sp, int64_t first, int64_t last) {
        return sp >= 0 && sp < SP_N && first >= 0 && last >= first && last < size[sp];
    };
    auto bad = [](const char* what) {
        set_error(std::string("internal: plan table out of range (") + what + ")");
        return HX_EINVAL;
    };
    for (const std::vector<Launch>* seq : {&P.prep, &P.apply, &P.diag_gemm})
        for (const Launch& L : *seq) {
            const bool ta = L.kind == TN_, tb = L.kind == NT;
            for (int64_t t = L.tile0; t < L.tile0 + L.ntile; ++t) {
                const Tile& tl = P.tiles[(size_t)t];
                if (tl.m <= 0 || tl.n <= 0) continue;
                if (tl.m > shape_rows(L.shape) || tl.n > shape_cols(L.shape)) return bad("tile extent");
                if (!inside(tl.cspace(), tl.coff, tl.coff + (int64_t)(tl.m - 1) * tl.ldc + tl.n - 1))
                    return bad("tile output");
                if (tl.tbeg < 0 || tl.tend < tl.tbeg || tl.tend > (int64_t)P.tasks.size()) return bad("task range");
                int64_t kt = 0;
                for (int j = tl.tbeg; j < tl.tend; ++j) {
                    const Task& k = P.tasks[(size_t)j];
                    kt += kpad(k.k, P.kstage);
                    if (k.k <= 0) continue;
                    const int64_t r1 = tl.r0 + tl.m - 1, c1 = tl.c0 + tl.n - 1;
                    const int64_t a0 = k.aoff + (ta ? tl.r0 : (int64_t)tl.r0 * k.lda);
                    const int64_t a1 = k.aoff + (ta ? (int64_t)(k.k - 1) * k.lda + r1 : r1 * k.lda + k.k - 1);
                    const int64_t b0 = k.boff + (tb ? (int64_t)tl.c0 * k.ldb : tl.c0);
                    const int64_t b1 = k.boff + (tb ? c1 * k.ldb + k.k - 1 : (int64_t)(k.k - 1) * k.ldb + c1);
                    if (!inside(k.aspace(), a0, a1)) return bad("A operand");
                    if (!inside(k.bspace(), b0, b1)) return bad("B operand");
                }
                if (kt != tl.ktot) return bad("tile depth");
            }
            for (int64_t r = L.red0; r < L.red0 + L.nred; ++r) {
                const Reduce& rd = P.reduces[(size_t)r];
                if (rd.m <= 0 || rd.n <= 0) continue;
                if (!inside(rd.cspace, rd.coff, rd.coff + (int64_t)(rd.m - 1) * rd.ldc + rd.n - 1))
                    return bad("reduction output");
                if (!inside(SP_PART, rd.pbase, rd.pbase + (int64_t)(rd.np - 1) * TM * TN +
                                                   (int64_t)(rd.m - 1) * rd.pld + rd.n - 1))
                    return bad("reduction partials");
            }
        }
    return HX_OK;
}

static void finalize_tables(Plan& P);
// XCD ordering of every recorded launch.  Each range is reordered in place and
// ranges are disjoint, so large plans spread them over host threads (largest
// first); the result does not depend on the thread count.
static void run_tile_sorts(Plan& P) {
    auto& R = P.sort_ranges;
    int64_t total = 0;
    for (auto& r : R) total += r.second;
    std::vector<size_t> ord(R.size());
    std::iota(ord.begin(), ord.end(), (size_t)0);
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return R[a].second > R[b].second; });
    std::atomic<size_t> next{0};
    auto work = [&]() {
        for (size_t j; (j = next.fetch_add(1)) < ord.size();) sort_tiles(P, R[ord[j]].first, R[ord[j]].second);
    };
    unsigned hw = std::thread::hardware_concurrency();
    int nth = (int)std::min<size_t>({R.size(), (size_t)16, (size_t)std::max(1u, hw)});
    if (total < 32768 || nth <= 1) {
        work();
    } else {
        std::vector<std::thread> pool;
        for (int i = 1; i < nth; ++i) pool.emplace_back(work);
        work();
        for (auto& t : pool) t.join();
    }
    R.clear();
}

static void finalize_tables(Plan& P) {
    run_tile_sorts(P);
    auto al = [](int64_t x) { return (x + 255) & ~(int64_t)255; };
    int64_t o = 0;
    P.off_tiles = o;
    o = al(o + (int64_t)P.tiles.size() * sizeof(Tile));
    P.off_tasks = o;
    o = al(o + (int64_t)P.tasks.size() * sizeof(Task));
    P.off_gathers = o;
    o = al(o + (int64_t)P.gathers.size() * sizeof(Gather));
    P.off_coef = o;
    o = al(o + (int64_t)P.coef.size() * sizeof(double));
    P.off_reduces = o;
    o = al(o + (int64_t)P.reduces.size() * sizeof(Reduce));
    P.table_bytes = std::max<int64_t>(o, 256);
}


// ---------------------------------------------------------------- batching

// Merge independent sigma-vector plans into one plan whose every stage is a
// single launch over all instances.  Instance i's operands live at its offsets
// in concatenated buffers (psi/sigma, L, R, workspace, coefficient table).
static int merge_plans(const std::vector<const Plan*>& in, Plan& M) {
    M.kind = PK_HEFF;
    M.n_chunks = 1;
    M.variant = in.empty() ? 0 : in[0]->variant;
    M.kstage = in.empty() ? 16 : in[0]->kstage;
    M.n_roots = in.empty() ? 1 : in[0]->n_roots;
    std::vector<std::array<int64_t, SP_N>> off(in.size());
    int64_t o_psi = 0, o_L = 0, o_R = 0, o_ws = 0, o_tab = 0;
    for (size_t i = 0; i < in.size(); ++i) {
        const Plan& P = *in[i];
        if (P.n_roots != in[0]->n_roots) {
            set_error("plan_batch: instances have different n_roots");
            return HX_EUNSUP;
        }
        if (P.variant != M.variant) {
            set_error("plan_batch: instances use different kernel variants");
            return HX_EUNSUP;
        }
        if (P.kind != PK_HEFF) {
            set_error("plan_batch: every instance must be a sigma-vector plan");
            return HX_EUNSUP;
        }
        M.n_chunks = std::max(M.n_chunks, P.n_chunks);
        off[i].fill(0);
        off[i][SP_PSI] = off[i][SP_OUT] = o_psi;
        off[i][SP_L] = o_L;
        off[i][SP_R] = o_R;
        off[i][SP_WS] = o_ws;
        off[i][SP_TAB] = o_tab;
        off[i][SP_PART] = o_ws + P.part_base;  // partials become workspace offsets
        M.inst_psi.push_back(o_psi);
        M.inst_L.push_back(o_L);
        M.inst_R.push_back(o_R);
        for (const auto& r : P.mix_ranges) M.mix_ranges.push_back({o_ws + r.first, o_ws + r.second});
        o_psi += P.psi_nnz;
        o_L += P.in_nnz;
        o_R += P.in2_nnz;
        o_ws += P.ws_doubles;
        o_tab += (int64_t)P.coef.size();
        M.flops_apply += P.flops_apply;
        M.flops_useful = std::max(M.flops_useful, 0.0) + (P.flops_useful < 0 ? P.flops_apply : P.flops_useful);
        M.flops_prepare += P.flops_prepare;
        M.bytes_apply += P.bytes_apply;
        M.n_tasks_apply += P.n_tasks_apply;
        M.n_mixed += P.n_mixed;
    }
    M.psi_nnz = o_psi;
    M.in_nnz = o_L;
    M.in2_nnz = o_R;
    M.ws_doubles = o_ws;
    M.part_base = 0;
    M.mix_end = 0;
    for (size_t i = 0; i < in.size(); ++i) M.coef.insert(M.coef.end(), in[i]->coef.begin(), in[i]->coef.end());

    auto remap_space = [&](size_t i, int sp, int64_t off_in, int& sp_out) -> int64_t {
        sp_out = sp == SP_PART ? SP_WS : sp;
        return off_in + off[i][sp];
    };
    // Merge the instances' launch sequences round by round: each instance's launches
    // stay in their order; the next launches of all instances that share kind and tile
    // shape are merged into one (instances touch disjoint data, so only the order
    // within an instance matters).  Chunked instances (several intermediate chunks)
    // take part in as many rounds as they have launches.
    auto merge_seq = [&](std::vector<Launch> Plan::*seq, std::vector<Launch>& out) -> int {
        std::vector<size_t> pos(in.size(), 0);
        for (;;) {
            int lead = -1;
            for (size_t i = 0; i < in.size() && lead < 0; ++i)
                if (pos[i] < (in[i]->*seq).size()) lead = (int)i;
            if (lead < 0) break;
            const Launch& K0 = (in[lead]->*seq)[pos[lead]];
            Launch L;
            L.kind = K0.kind;
            L.shape = K0.shape;
            L.stage = (int)out.size();
            L.tile0 = (int64_t)M.tiles.size();
            L.flops = 0;
            std::vector<Reduce> reds;
            for (size_t i = 0; i < in.size(); ++i) {
                const Plan& P = *in[i];
                if (pos[i] >= (P.*seq).size()) continue;
                const Launch& S = (P.*seq)[pos[i]];
                if (S.kind != L.kind || S.shape != L.shape) continue;
                ++pos[i];
                L.flops += S.flops;
                const int32_t tbase = (int32_t)M.tasks.size();
                int32_t tmin = INT32_MAX, tmax = 0;
                for (int64_t t = S.tile0; t < S.tile0 + S.ntile; ++t) {
                    tmin = std::min(tmin, P.tiles[t].tbeg);
                    tmax = std::max(tmax, P.tiles[t].tend);
                }
                if (tmin > tmax) tmin = tmax = 0;
                for (int32_t j = tmin; j < tmax; ++j) {
                    Task t = P.tasks[j];
                    int a, b;
                    t.aoff = remap_space(i, t.spaces & 0xff, t.aoff, a);
                    t.boff = remap_space(i, (t.spaces >> 8) & 0xff, t.boff, b);
                    t.set_spaces(a, b);
                    M.tasks.push_back(t);
                }
                for (int64_t t = S.tile0; t < S.tile0 + S.ntile; ++t) {
                    Tile tl = P.tiles[t];
                    int c;
                    tl.coff = remap_space(i, tl.cspace(), tl.coff, c);
                    tl.set_out(c, tl.beta());
                    tl.tbeg = tl.tbeg - tmin + tbase;
                    tl.tend = tl.tend - tmin + tbase;
                    M.tiles.push_back(tl);
                }
                for (int64_t r = S.red0; r < S.red0 + S.nred; ++r) {
                    Reduce rd = P.reduces[r];
                    int c;
                    rd.coff = remap_space(i, rd.cspace, rd.coff, c);
                    rd.cspace = (int8_t)c;
                    rd.pbase += off[i][SP_PART];
                    reds.push_back(rd);
                }
            }
            L.ntile = (int64_t)M.tiles.size() - L.tile0;
            M.sort_ranges.push_back({L.tile0, L.ntile});
            L.red0 = (int64_t)M.reduces.size();
            L.nred = (int64_t)reds.size();
            M.reduces.insert(M.reduces.end(), reds.begin(), reds.end());
            if (L.ntile > 0 || L.nred > 0) out.push_back(L);
        }
        return HX_OK;
    };
    int rc;
    if ((rc = merge_seq(&Plan::prep, M.prep))) return rc;
    if ((rc = merge_seq(&Plan::apply, M.apply))) return rc;
    if ((rc = merge_seq(&Plan::diag_gemm, M.diag_gemm))) return rc;
    for (size_t i = 0; i < in.size(); ++i) {
        for (const FillLaunch& f : in[i]->diag_fill) {
            FillLaunch g = f;
            g.off += off[i][f.space];
            M.diag_fill.push_back(g);
        }
        // each gather list of the instance becomes one launch of the merged list
        auto copy_list = [&](const std::vector<GatherLaunch>& src, std::vector<GatherLaunch>& dst) {
            GatherLaunch gl;
            gl.g0 = (int64_t)M.gathers.size();
            for (const GatherLaunch& sl : src)
                for (int64_t q = sl.g0; q < sl.g0 + sl.ng; ++q) {
                    Gather g = in[i]->gathers[(size_t)q];
                    int a, b;
                    g.soff = remap_space(i, g.sspace, g.soff, a);
                    g.doff = remap_space(i, g.dspace, g.doff, b);
                    g.sspace = (int8_t)a;
                    g.dspace = (int8_t)b;
                    M.gathers.push_back(g);
                }
            gl.ng = (int64_t)M.gathers.size() - gl.g0;
            if (gl.ng) dst.push_back(gl);
        };
        copy_list(in[i]->diag_gather, M.diag_gather);
        copy_list(in[i]->prep_gather, M.prep_gather);
    }
    for (auto& L : M.apply) M.n_tiles_apply += L.ntile;
    if (!check_task_index_range(M)) return HX_EINVAL;
    return HX_OK;
}

}  // namespace hx

using namespace hx;

extern "C" {

const char* hx_last_error(void) { return g_err.c_str(); }

int hx_env_layout(const hx_bond* bond, const hx_opset* ops, int64_t* op_off, int64_t* blk_off) {
    Bond b;
    OpSet o;
    if (!parse_bond(bond, b, "env_layout") || !parse_ops(ops, o, "env_layout")) return HX_EINVAL;
    EnvLayout L = env_layout(b, o);
    if (op_off) std::copy(L.op_off.begin(), L.op_off.end(), op_off);
    if (blk_off) std::copy(L.blk_off.begin(), L.blk_off.end(), blk_off);
    return HX_OK;
}

int64_t hx_psi_layout(const hx_bond* lbond, const hx_bond* rbond, int64_t max_blocks, int32_t* keys,
                      int64_t* off) {
    Bond lb, rb;
    if (!parse_bond(lbond, lb, "psi_layout left") || !parse_bond(rbond, rb, "psi_layout right")) return HX_EINVAL;
    PsiLayout P = psi_layout(lb, rb);
    int64_t n = (int64_t)P.blocks.size();
    if (keys || off) {
        if (max_blocks < n) {
            set_error("psi_layout: max_blocks too small");
            return HX_EINVAL;
        }
        for (int64_t i = 0; i < n; ++i) {
            if (keys) {
                keys[4 * i] = P.blocks[i].il;
                keys[4 * i + 1] = P.blocks[i].s1;
                keys[4 * i + 2] = P.blocks[i].s2;
                keys[4 * i + 3] = P.blocks[i].ir;
            }
            if (off) off[i] = P.blocks[i].off;
        }
        if (off) off[n] = P.nnz;
    }
    return n;
}

int64_t hx_site_layout(const hx_bond* lbond, const hx_bond* rbond, int64_t max_blocks, int32_t* keys,
                       int64_t* off) {
    Bond lb, rb;
    if (!parse_bond(lbond, lb, "site_layout left") || !parse_bond(rbond, rb, "site_layout right"))
        return HX_EINVAL;
    SiteLayout S = site_layout(lb, rb);
    int64_t n = (int64_t)S.blocks.size();
    if (keys || off) {
        if (max_blocks < n) {
            set_error("site_layout: max_blocks too small");
            return HX_EINVAL;
        }
        for (int64_t i = 0; i < n; ++i) {
            if (keys) {
                keys[3 * i] = S.blocks[i].il;
                keys[3 * i + 1] = S.blocks[i].s;
                keys[3 * i + 2] = S.blocks[i].ir;
            }
            if (off) off[i] = S.blocks[i].off;
        }
        if (off) off[n] = S.nnz;
    }
    return n;
}

// Runs a plan build; a C++ exception (host memory exhausted, or an internal
// failure) becomes an error code and message instead of crossing the C ABI.
extern "C++" {
template <typename F>
static int guarded(F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        set_error("out of host memory while building the plan");
        return HX_EINVAL;
    } catch (const std::exception& e) {
        set_error(std::string("internal: ") + e.what());
        return HX_EINVAL;
    }
}
}

int hx_heff_plan_create(const hx_bond* lbond, const hx_bond* rbond, const hx_opset* Lops, const hx_opset* mid,
                        const hx_opset* Rops, const hx_mpo_site* W1, const hx_mpo_site* W2,
                        const hx_plan_opts* opts, hx_plan** out) {
    if (!out) {
        set_error("heff_plan_create: null output");
        return HX_EINVAL;
    }
    *out = nullptr;
    Bond lb, rb;
    OpSet Lo, Mo, Ro;
    if (!parse_bond(lbond, lb, "heff left bond") || !parse_bond(rbond, rb, "heff right bond")) return HX_EINVAL;
    if (!parse_ops(Lops, Lo, "heff Lops") || !parse_ops(mid, Mo, "heff mid") || !parse_ops(Rops, Ro, "heff Rops"))
        return HX_EINVAL;
    std::vector<Entry> e1, e2;
    if (!parse_mpo(W1, Lo, Mo, true, e1, "heff W1") || !parse_mpo(W2, Mo, Ro, false, e2, "heff W2"))
        return HX_EINVAL;
    Plan* P = new Plan();
    int rc = guarded([&] {
        int r = build_heff(*P, lb, rb, Lo, Mo, Ro, e1, e2, opts);
        if (r == HX_OK) r = check_gemm_bounds(*P);
        if (r == HX_OK) finalize_tables(*P);
        return r;
    });
    if (rc != HX_OK) {
        delete P;
        return rc;
    }
    *out = reinterpret_cast<hx_plan*>(P);
    return HX_OK;
}

int hx_heff1_plan_create(const hx_bond* lbond, const hx_bond* rbond, const hx_opset* Lops, const hx_opset* Rops,
                         const hx_mpo_site* W, const hx_plan_opts* opts, hx_plan** out) {
    if (!out) {
        set_error("heff1_plan_create: null output");
        return HX_EINVAL;
    }
    *out = nullptr;
    Bond lb, rb;
    OpSet Lo, Ro;
    if (!parse_bond(lbond, lb, "heff1 left bond") || !parse_bond(rbond, rb, "heff1 right bond")) return HX_EINVAL;
    if (!parse_ops(Lops, Lo, "heff1 Lops") || !parse_ops(Rops, Ro, "heff1 Rops")) return HX_EINVAL;
    std::vector<Entry> e1;
    if (!parse_mpo(W, Lo, Ro, true, e1, "heff1 W")) return HX_EINVAL;
    Plan* P = new Plan();
    int rc = guarded([&] {
        int r = build_heff(*P, lb, rb, Lo, Ro, Ro, e1, {}, opts, true);
        if (r == HX_OK) r = check_gemm_bounds(*P);
        if (r == HX_OK) finalize_tables(*P);
        return r;
    });
    if (rc != HX_OK) {
        delete P;
        return rc;
    }
    *out = reinterpret_cast<hx_plan*>(P);
    return HX_OK;
}

int64_t hx_psi1_layout(const hx_bond* lbond, const hx_bond* rbond, int64_t max_blocks, int32_t* keys,
                       int64_t* off) {
    Bond lb, rb;
    if (!parse_bond(lbond, lb, "psi1_layout left bond") || !parse_bond(rbond, rb, "psi1_layout right bond"))
        return HX_EINVAL;
    PsiLayout P = psi_layout(lb, rb, true);
    const int64_t n = (int64_t)P.blocks.size();
    if (keys && off) {
        if (max_blocks < n) {
            set_error("psi1_layout: max_blocks too small");
            return HX_EINVAL;
        }
        for (int64_t i = 0; i < n; ++i) {
            keys[3 * i] = P.blocks[i].il;
            keys[3 * i + 1] = P.blocks[i].s1;
            keys[3 * i + 2] = P.blocks[i].ir;
            off[i] = P.blocks[i].off;
        }
        off[n] = P.nnz;
    }
    return n;
}

int hx_heff_vjp_plan_create(const hx_bond* lbond, const hx_bond* rbond, const hx_opset* Lops, const hx_opset* mid,
                            const hx_opset* Rops, const hx_mpo_site* W1, const hx_mpo_site* W2,
                            const hx_plan_opts* opts, hx_plan** out) {
    if (!out) {
        set_error("heff_vjp_plan_create: null output");
        return HX_EINVAL;
    }
    *out = nullptr;
    Bond lb, rb;
    OpSet Lo, Mo, Ro;
    if (!parse_bond(lbond, lb, "vjp left bond") || !parse_bond(rbond, rb, "vjp right bond")) return HX_EINVAL;
    if (!parse_ops(Lops, Lo, "vjp Lops") || !parse_ops(mid, Mo, "vjp mid") || !parse_ops(Rops, Ro, "vjp Rops"))
        return HX_EINVAL;
    std::vector<Entry> e1, e2;
    if (!parse_mpo(W1, Lo, Mo, true, e1, "vjp W1") || !parse_mpo(W2, Mo, Ro, false, e2, "vjp W2")) return HX_EINVAL;
    Plan* P = new Plan();
    int rc = guarded([&] {
        int r = build_heff_vjp(*P, lb, rb, Lo, Mo, Ro, e1, e2, opts);
        if (r == HX_OK) r = check_gemm_bounds(*P);
        if (r == HX_OK) finalize_tables(*P);
        return r;
    });
    if (rc != HX_OK) {
        delete P;
        return rc;
    }
    *out = reinterpret_cast<hx_plan*>(P);
    return HX_OK;
}

int hx_heff1_vjp_plan_create(const hx_bond* lbond, const hx_bond* rbond, const hx_opset* Lops, const hx_opset* Rops,
                             const hx_mpo_site* W, const hx_plan_opts* opts, hx_plan** out) {
    if (!out) {
        set_error("heff1_vjp_plan_create: null output");
        return HX_EINVAL;
    }
    *out = nullptr;
    Bond lb, rb;
    OpSet Lo, Ro;
    if (!parse_bond(lbond, lb, "vjp1 left bond") || !parse_bond(rbond, rb, "vjp1 right bond")) return HX_EINVAL;
    if (!parse_ops(Lops, Lo, "vjp1 Lops") || !parse_ops(Rops, Ro, "vjp1 Rops")) return HX_EINVAL;
    std::vector<Entry> e1;
    if (!parse_mpo(W, Lo, Ro, true, e1, "vjp1 W")) return HX_EINVAL;
    Plan* P = new Plan();
    int rc = guarded([&] {
        int r = build_heff_vjp(*P, lb, rb, Lo, Ro, Ro, e1, {}, opts, true);
        if (r == HX_OK) r = check_gemm_bounds(*P);
        if (r == HX_OK) finalize_tables(*P);
        return r;
    });
    if (rc != HX_OK) {
        delete P;
        return rc;
    }
    *out = reinterpret_cast<hx_plan*>(P);
    return HX_OK;
}

int hx_env_plan_create(int direction, const hx_bond* bond_in, const hx_bond* bond_out, const hx_opset* ops_in,
                       const hx_opset* ops_out, const hx_mpo_site* W, const hx_plan_opts* opts, hx_plan** out) {
    if (!out || (direction != 0 && direction != 1)) {
        set_error("env_plan_create: bad direction or null output");
        return HX_EINVAL;
    }
    *out = nullptr;
    Bond bi, bo;
    OpSet oi, oo;
    if (!parse_bond(bond_in, bi, "env bond_in") || !parse_bond(bond_out, bo, "env bond_out")) return HX_EINVAL;
    if (!parse_ops(ops_in, oi, "env ops_in") || !parse_ops(ops_out, oo, "env ops_out")) return HX_EINVAL;
    std::vector<Entry> ents;
    bool ok = direction == 0 ? parse_mpo(W, oi, oo, true, ents, "env W") : parse_mpo(W, oo, oi, false, ents, "env W");
    if (!ok) return HX_EINVAL;
    Plan* P = new Plan();
    int rc = guarded([&] {
        int r = build_env(*P, direction, bi, bo, oi, oo, ents, opts);
        if (r == HX_OK) r = check_gemm_bounds(*P);
        if (r == HX_OK) finalize_tables(*P);
        return r;
    });
    if (rc != HX_OK) {
        delete P;
        return rc;
    }
    *out = reinterpret_cast<hx_plan*>(P);
    return HX_OK;
}

int hx_heff_plan_batch(const hx_plan* const* plans, int32_t n, hx_plan** out) {
    if (!out || !plans || n < 1) {
        set_error("plan_batch: bad arguments");
        return HX_EINVAL;
    }
    *out = nullptr;
    std::vector<const Plan*> in;
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) {
            set_error("plan_batch: null instance plan");
            return HX_EINVAL;
        }
        in.push_back(reinterpret_cast<const Plan*>(plans[i]));
    }
    Plan* M = new Plan();
    int rc = guarded([&] {
        int r = merge_plans(in, *M);
        if (r == HX_OK) r = check_gemm_bounds(*M);
        if (r == HX_OK) finalize_tables(*M);
        return r;
    });
    if (rc != HX_OK) {
        delete M;
        return rc;
    }
    *out = reinterpret_cast<hx_plan*>(M);
    return HX_OK;
}

int hx_batch_offsets(const hx_plan* plan, int32_t i, int64_t* psi_off, int64_t* L_off, int64_t* R_off) {
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if (!P || i < 0 || (size_t)i >= P->inst_psi.size()) {
        set_error("batch_offsets: not a batched plan or instance out of range");
        return HX_EINVAL;
    }
    if (psi_off) *psi_off = P->inst_psi[i];
    if (L_off) *L_off = P->inst_L[i];
    if (R_off) *R_off = P->inst_R[i];
    return HX_OK;
}

int hx_plan_get_info(const hx_plan* plan, hx_plan_info* info) {
    if (!plan || !info) {
        set_error("plan_info: null argument");
        return HX_EINVAL;
    }
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    info->psi_nnz = P->psi_nnz;
    info->in_nnz = P->in_nnz;
    info->in2_nnz = P->in2_nnz;
    info->out_nnz = P->out_nnz;
    info->table_bytes = P->table_bytes;
    info->ws_bytes = std::max<int64_t>(P->ws_doubles * 8, 256);
    info->flops_apply = P->flops_apply;
    info->flops_useful = P->flops_useful < 0 ? P->flops_apply : P->flops_useful;
    info->flops_prepare = P->flops_prepare;
    info->bytes_apply = P->bytes_apply;
    info->n_tasks = P->n_tasks_apply;
    info->n_tiles = P->n_tiles_apply;
    info->n_chunks = P->n_chunks;
    info->n_mixed = P->n_mixed;
    return HX_OK;
}

void hx_plan_destroy(hx_plan* plan) { delete reinterpret_cast<Plan*>(plan); }

}  // extern "C"
