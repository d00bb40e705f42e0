// Host side of the AC evaluation library: blob parsing and validation,
// derived down-pass structures, workspace layout, argument checks and the
// extern "C" entry points declared in include/qkc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include "qkc.h"
#include "qkc_internal.h"

namespace qkc {

template <typename T>
hipError_t launch_fixed_slots(const DevGraph &g, const double *noise, void *wfix, hipStream_t st);
template <typename T>
hipError_t launch_eval(const DevGraph &g, const SopPlan &sp, int grid, int block, const double *theta, const int32_t *param_of, int P,
                       const uint64_t *evidence, int64_t B, const void *wfix, void *vals, size_t per_wg_elems,
                       void *amp_out, double *prob_out, hipStream_t st);
template <typename T>
hipError_t launch_grad(const DevGraph &g, const SopPlan &sp, int grid, int block, const double *theta, const int32_t *param_of,
                       const uint64_t *evidence, int64_t B, const void *wfix, void *vals, size_t per_wg_elems,
                       int mode, const void *cotangent, const double *weight, double *contrib, int P,
                       double *grad, void *amp_out, void *dfdtheta_out, void *dind_out, void *sort_ws,
                       size_t sort_ws_bytes, hipStream_t st);
size_t grad_sort_bytes(int64_t B);
template <typename T>
hipError_t launch_sample(const DevGraph &g, int grid, const double *theta, const void *wfix, void *vals,
                         size_t per_wg_elems, const SampleArgs &a, hipStream_t st);
size_t lds_bytes(const DevGraph &g);
template <typename T>
size_t sample_lds_chain_bytes(const DevGraph &g, const LdsPlan &lp);
size_t sample_lds_meta_bytes(const LdsPlan &lp);
template <typename T>
hipError_t launch_sample_stream(const DevGraph &g, const SopPlan &sp, int grid, int block, const double *theta,
                                const void *wfix, void *vals, size_t per_wg_elems, const SampleArgs &a,
                                hipStream_t st);
template <typename T>
hipError_t launch_sample_lds(const DevGraph &g, const LdsPlan &lp, int cpw, int wpc, int grid, const double *theta,
                             const double *noise, const SampleArgs &a, hipStream_t st);
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t st);
size_t mpe_lds_bytes(const DevGraph &g);
hipError_t launch_mpe(const DevGraph &g, const MpePlan &mp, int grid, int block, const double *theta,
                      const int32_t *param_of, int P, const uint64_t *evidence, int64_t B, const void *wfix,
                      void *vals, size_t per_wg_elems, double *prob_out, uint64_t *mpe_out, hipStream_t st);
hipError_t static_scratch_address(void **out);
template <typename T>
int resident_blocks(const DevGraph &g, const SopPlan &sp, int which, int block);

}  // namespace qkc

using namespace qkc;

static_assert(AC_STATIC_SCRATCH_BYTES == STATIC_SCRATCH_BYTES, "static scratch size in qkc.h and the library agree");

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

static ac_status fail(ac_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

static ac_status fail_hip(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(AC_ERR_OOM, "%s: %s", what, hipGetErrorString(e));
    return fail(AC_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// library-owned scratch of ac_eval_batch_static, one address per device
// ---------------------------------------------------------------------------

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Resolve this device's copy of the scratch array once (the device must be
// current).  Later calls return the stored address.
hipError_t resolve_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = static_scratch_address(&ptr);
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

void *scratch_of(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace

// ---------------------------------------------------------------------------
// graph handle
// ---------------------------------------------------------------------------

struct ac_graph {
    DevGraph dev;
    LdsPlan plan{};
    bool has_plan = false;
    SopPlan sop{};
    bool has_sop = false;
    std::vector<uint32_t> plan_level_ptr;   // host copy (launch heuristics)
    void *dmem = nullptr;
    int device = 0;
    int n_cu = 0;
    int resident[2][4] = {{1, 1, 1, 1}, {1, 1, 1, 1}};   // [dtype][eval, grad, sample, stream] per CU
    int stream_waves = 0;                                 // forced waves per streaming workgroup (0: per call)
    int tile_waves = 0;                                   // forced waves per upward/gradient/max-product workgroup (0: per call)
    int wide_resident[2][4][3] = {};                      // [dtype][eval, grad, -, stream][4, 8, 16 waves] per CU
    ac_info_t info{};
    std::vector<uint8_t> var_dom;
    std::vector<uint32_t> var_offset;
    MpePlan mpe{};
    std::string mpe_why;                                  // why ac_mpe_batch refuses this AC ("" if it does not)
};

namespace {

struct Reader {
    const uint8_t *base;
    size_t n, pos = 0;
    bool ok = true;
    template <typename T>
    const T *take(size_t count) {
        pos = (pos + 7) & ~static_cast<size_t>(7);
        size_t bytes = count * sizeof(T);
        if (pos > n || bytes > n - pos) {
            ok = false;
            return nullptr;
        }
        const T *p = reinterpret_cast<const T *>(base + pos);
        pos += bytes;
        return p;
    }
    // arrays packed without alignment padding between them
    template <typename T>
    const T *take_packed(size_t count) {
        size_t bytes = count * sizeof(T);
        if (pos > n || bytes > n - pos) {
            ok = false;
            return nullptr;
        }
        const T *p = reinterpret_cast<const T *>(base + pos);
        pos += bytes;
        return p;
    }
};

const uint8_t MAGIC[8] = {'Q', 'K', 'C', 'A', 'C', 0, 0, 1};

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

int cdiv64(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// Node-parallel plan (see LdsPlan in qkc_internal.h), built on the host.
struct HostPlan {
    std::vector<uint64_t> fwd, orec, edg, fwd_u, edg_u, dterm;
    std::vector<uint32_t> level_ptr, level_prod, brec, estart, dstart, esel;
    uint32_t N = 0, L = 0, root = 0, max_edges = 0;
    bool ok = false;
};

uint32_t encode_leaf(uint32_t r, const std::vector<uint32_t> &var_field) {
    if ((r >> 30) != TAG_IND) return r;
    const uint32_t x = r & REF_MASK, v = x & 0xffffffu, u = x >> 24, fld = var_field[v];
    return dev_ind_ref(u, (fld & 3u) + 1u, fld >> 8, (fld >> 2) & 63u);
}

HostPlan build_plan(uint32_t N, const uint8_t *op, const uint32_t *row_ptr, const uint32_t *col, uint32_t root,
                    const std::vector<uint32_t> &ind_base, const std::vector<uint32_t> &var_field, uint32_t n_ind,
                    uint32_t n_sel, uint32_t n_slots, const std::vector<uint32_t> &sel_dev,
                    const std::vector<uint32_t> &vsel_ptr, const std::vector<uint32_t> &vsel) {
    HostPlan P;
    struct PN {
        uint8_t op;
        uint32_t a, b;       // node refs hold pre-sort plan ids (tag 0); leaves keep blob refs
    };
    std::vector<PN> nodes;
    nodes.reserve(2 * static_cast<size_t>(N));
    std::vector<uint32_t> map(N), kids, next;
    auto make = [&](uint8_t o, uint32_t a, uint32_t b) {
        nodes.push_back(PN{o, a, b});
        return static_cast<uint32_t>(nodes.size() - 1);
    };
    for (uint32_t i = 0; i < N; ++i) {
        kids.clear();
        for (uint32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const uint32_t r = col[e];
            kids.push_back((r >> 30) == TAG_NODE ? map[r & REF_MASK] : r);
        }
        if (kids.size() == 1) {
            map[i] = make(op[i], kids[0], IDENT_REF);
        } else if (op[i] == 1) {                       // product: chain
            uint32_t cur = make(1, kids[0], kids[1]);
            for (size_t j = 2; j < kids.size(); ++j) cur = make(1, cur, kids[j]);
            map[i] = cur;
        } else {                                       // sum: balanced tree
            while (kids.size() > 2) {
                next.clear();
                for (size_t j = 0; j + 1 < kids.size(); j += 2) next.push_back(make(0, kids[j], kids[j + 1]));
                if (kids.size() % 2) next.push_back(kids.back());
                kids.swap(next);
            }
            map[i] = make(0, kids[0], kids[1]);
        }
    }
    const uint32_t M = static_cast<uint32_t>(nodes.size());
    const uint32_t proot = map[root];
    auto is_node = [](uint32_t r) { return r != IDENT_REF && (r >> 30) == TAG_NODE; };
    std::vector<uint32_t> lev(M), fan(M, 0);
    uint32_t Lmax = 0;
    for (uint32_t n = 0; n < M; ++n) {
        uint32_t l = 0;
        if (is_node(nodes[n].a)) l = std::max(l, lev[nodes[n].a]), fan[nodes[n].a]++;
        if (is_node(nodes[n].b)) l = std::max(l, lev[nodes[n].b]), fan[nodes[n].b]++;
        lev[n] = l + 1;
        Lmax = std::max(Lmax, lev[n]);
    }
    uint32_t at_top = 0;
    for (uint32_t n = 0; n < M; ++n) at_top += lev[n] == Lmax;
    if (at_top != 1 || lev[proot] != Lmax) return P;          // unreachable nodes: no plan
    std::vector<uint32_t> order(M), newid(M);
    for (uint32_t n = 0; n < M; ++n) order[n] = n;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        if (lev[x] != lev[y]) return lev[x] < lev[y];
        if (nodes[x].op != nodes[y].op) return nodes[x].op < nodes[y].op;
        return fan[x] < fan[y];
    });
    for (uint32_t j = 0; j < M; ++j) newid[order[j]] = j;
    auto plan_ref = [&](uint32_t r) -> uint32_t {
        if (r == IDENT_REF) return IDENT_REF;
        return (r >> 30) == TAG_NODE ? newid[r] : encode_leaf(r, var_field);
    };
    P.fwd.resize(M);
    P.level_ptr.assign(Lmax + 1, 0);
    P.level_prod.assign(Lmax, 0);
    std::vector<uint32_t> n_sum(Lmax + 1, 0);
    for (uint32_t j = 0; j < M; ++j) {
        const PN &nd = nodes[order[j]];
        P.fwd[j] = static_cast<uint64_t>(plan_ref(nd.a)) | (static_cast<uint64_t>(plan_ref(nd.b)) << 32);
        P.level_ptr[lev[order[j]]]++;
        if (nd.op == 0) n_sum[lev[order[j]]]++;
    }
    for (uint32_t l = 1; l <= Lmax; ++l) P.level_ptr[l] += P.level_ptr[l - 1];
    for (uint32_t l = 0; l < Lmax; ++l) P.level_prod[l] = P.level_ptr[l] + n_sum[l + 1];
    // parent edges of nodes, indicator leaves and selectors, in increasing
    // parent order; selector targets follow the per-variable selector lists
    // (vsel), so the selectors of one variable are contiguous targets
    const size_t T = static_cast<size_t>(M) + n_ind + n_sel;
    std::vector<uint32_t> selpos(n_sel, 0);
    for (uint32_t k = 0; k < n_sel; ++k) selpos[vsel[k]] = k;
    std::vector<std::vector<uint64_t>> edges(T);
    auto target_of = [&](uint32_t r) -> int64_t {
        if (r == IDENT_REF) return -1;
        const uint32_t tag = r >> 30;
        if (tag == TAG_NODE) return newid[r];
        if (tag == TAG_IND) {
            const uint32_t x = r & REF_MASK;
            return static_cast<int64_t>(M) + ind_base[x & 0xffffffu] + (x >> 24);
        }
        if (tag == TAG_SEL) return static_cast<int64_t>(M) + n_ind + selpos[r & REF_MASK];
        return -1;
    };
    for (uint32_t j = 0; j < M; ++j) {
        const PN &nd = nodes[order[j]];
        const uint32_t ch[2] = {nd.a, nd.b};
        for (int t = 0; t < 2; ++t) {
            const int64_t tg = target_of(ch[t]);
            if (tg < 0) continue;
            uint32_t sib = NO_SIBLING;
            if (nd.op == 1 && ch[1 - t] != IDENT_REF) sib = plan_ref(ch[1 - t]);
            edges[tg].push_back(static_cast<uint64_t>(j) | (static_cast<uint64_t>(sib) << 32));
        }
    }
    P.estart.assign(T + 1, 0);
    for (size_t t = 0; t < T; ++t) {
        P.estart[t + 1] = P.estart[t] + static_cast<uint32_t>(edges[t].size());
        P.edg.insert(P.edg.end(), edges[t].begin(), edges[t].end());
    }
    for (uint32_t k = 0; k < n_sel; ++k)
        P.esel.insert(P.esel.end(), edges[static_cast<size_t>(M) + n_ind + k].size(), vsel[k]);
    for (uint32_t l = 0; l < Lmax; ++l)
        P.max_edges = std::max(P.max_edges, P.estart[P.level_ptr[l + 1]] - P.estart[P.level_ptr[l]]);
    P.max_edges = std::max(P.max_edges, P.estart[T] - P.estart[M]);
    P.brec.assign(4 * T, 0);
    for (size_t t = 0; t < T; ++t) {
        const auto &ev = edges[t];
        P.brec[4 * t + 0] = static_cast<uint32_t>(ev.size());
        P.brec[4 * t + 1] = static_cast<uint32_t>(P.orec.size());
        P.brec[4 * t + 2] = ev.empty() ? 0u : static_cast<uint32_t>(ev[0]);
        P.brec[4 * t + 3] = ev.empty() ? NO_SIBLING : static_cast<uint32_t>(ev[0] >> 32);
        for (size_t q = 1; q < ev.size(); ++q) P.orec.push_back(ev[q]);
    }
    // unified references for the LDS kernel: [node | slot | selector]
    auto unify = [&](uint32_t r) -> uint32_t {
        if (r == IDENT_REF || r == NO_SIBLING) return r;
        const uint32_t tag = r >> 30, x = r & REF_MASK;
        if (tag == TAG_SLOT) return M + x;
        if (tag == TAG_SEL) return M + n_slots + x;
        return r;                                   // node index (tag 0) or indicator (tag 1)
    };
    P.fwd_u.resize(M);
    for (uint32_t j = 0; j < M; ++j) {
        const uint64_t f = P.fwd[j];
        const uint32_t a = unify(static_cast<uint32_t>(f)), b = unify(static_cast<uint32_t>(f >> 32));
        P.fwd_u[j] = static_cast<uint64_t>(a) | (static_cast<uint64_t>(b) << 32);
    }
    P.edg_u.resize(P.edg.size());
    for (size_t e = 0; e < P.edg.size(); ++e) {
        const uint64_t rr = P.edg[e];
        P.edg_u[e] = (rr & 0xffffffffull) | (static_cast<uint64_t>(unify(static_cast<uint32_t>(rr >> 32))) << 32);
    }
    // d root / d lambda terms per indicator: its own leaf edges, and every
    // leaf edge of the selectors of its variable times the selector's weight
    const uint32_t leaf0 = P.estart[M];
    P.dstart.assign(n_ind + 1, 0);
    for (uint32_t v = 0; v + 1 < ind_base.size(); ++v) {
        for (uint32_t u = 0; u < ind_base[v + 1] - ind_base[v]; ++u) {
            const uint32_t t = ind_base[v] + u;
            for (uint32_t e = P.estart[M + t]; e < P.estart[M + t + 1]; ++e)
                P.dterm.push_back(static_cast<uint64_t>(e - leaf0) | (static_cast<uint64_t>(NO_SLOT) << 32));
            for (uint32_t qq = vsel_ptr[v]; qq < vsel_ptr[v + 1]; ++qq) {
                const uint32_t q = vsel[qq];
                const uint32_t sl = u < static_cast<uint32_t>(SEL_DOM) ? sel_dev[static_cast<size_t>(q) * SEL_REC + 1 + u]
                                                                       : NO_SLOT;
                if (sl == NO_SLOT) continue;
                for (uint32_t e = P.estart[M + n_ind + qq]; e < P.estart[M + n_ind + qq + 1]; ++e)
                    P.dterm.push_back(static_cast<uint64_t>(e - leaf0) | (static_cast<uint64_t>(sl) << 32));
            }
            P.dstart[t + 1] = static_cast<uint32_t>(P.dterm.size());
        }
    }
    P.N = M;
    P.L = Lmax;
    P.root = newid[proot];
    P.ok = true;
    return P;
}

// Sum-of-products plan (see SopPlan in qkc_internal.h), built on the host.
struct HostSop {
    std::vector<uint32_t> level_ptr, fptr, ostart, occ, osel;
    std::vector<uint64_t> frec, frec_live;
    std::vector<uint32_t> srow;
    uint32_t S = 0, L = 0, root = 0, max_factors = 0, live_rows = 0;
    uint64_t node_factors = 0, down_reads = 0, leaf_reads = 0;   // row counts of the streaming model
    uint32_t max_sib = 0;      // most siblings of an occurrence of a super-node or leaf target
    bool ok = false;
};

HostSop build_sop(uint32_t N, const uint8_t *op, const uint32_t *row_ptr, const uint32_t *col, uint32_t root,
                  const std::vector<uint32_t> &ind_base, const std::vector<uint32_t> &var_field, uint32_t n_ind,
                  uint32_t n_sel, const std::vector<uint32_t> &vsel, uint32_t n_angle_slots) {
    HostSop P;
    // parents of each node: a product with exactly one parent, a sum, is folded into it
    std::vector<uint32_t> npar(N, 0), parent(N, 0);
    for (uint32_t i = 0; i < N; ++i)
        for (uint32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if ((col[e] >> 30) == TAG_NODE) {
                const uint32_t c = col[e] & REF_MASK;
                npar[c]++;
                parent[c] = i;
            }
    std::vector<uint8_t> folded(N, 0);
    for (uint32_t i = 0; i < N; ++i)
        folded[i] = op[i] == 1 && npar[i] == 1 && i != root && op[parent[i]] == 0;
    // super-nodes (pre-sort ids): terms as factor lists; node refs hold pre-sort super ids (tag 0)
    struct SN {
        std::vector<std::vector<uint32_t>> terms;
        std::vector<uint8_t> direct;           // per term: a sum's own (non-product) child
    };
    std::vector<SN> sn;
    sn.reserve(N);
    std::vector<uint32_t> sid(N, 0xFFFFFFFFu);
    bool bad = false;
    auto fref = [&](uint32_t r) -> uint32_t {
        if ((r >> 30) != TAG_NODE) return r;
        const uint32_t x = sid[r & REF_MASK];
        if (x == 0xFFFFFFFFu) bad = true;                      // a folded or later node: no plan
        return x & REF_MASK;
    };
    // a term of more than SOP_MAX_FACTORS factors: its leading factors become a
    // product super-node (multiplied in the same order)
    auto cap_term = [&](std::vector<uint32_t> t) {
        while (t.size() > static_cast<size_t>(SOP_MAX_FACTORS)) {
            SN x;
            x.terms.emplace_back(t.begin(), t.begin() + SOP_MAX_FACTORS);
            x.direct.push_back(0);
            sn.push_back(std::move(x));
            std::vector<uint32_t> rest;
            rest.push_back(static_cast<uint32_t>(sn.size() - 1));
            rest.insert(rest.end(), t.begin() + SOP_MAX_FACTORS, t.end());
            t.swap(rest);
        }
        return t;
    };
    for (uint32_t i = 0; i < N; ++i) {
        if (folded[i]) continue;
        if (row_ptr[i + 1] <= row_ptr[i]) return P;               // a node without children
        std::vector<std::vector<uint32_t>> terms;
        std::vector<uint8_t> direct;
        if (op[i] == 0) {
            for (uint32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                const uint32_t r = col[e];
                if ((r >> 30) == TAG_NODE && folded[r & REF_MASK]) {
                    const uint32_t c = r & REF_MASK;
                    if (row_ptr[c + 1] <= row_ptr[c]) return P;
                    std::vector<uint32_t> t;
                    for (uint32_t f = row_ptr[c]; f < row_ptr[c + 1]; ++f) {
                        if ((col[f] >> 30) == TAG_NODE && folded[col[f] & REF_MASK]) return P;   // not below a sum
                        t.push_back(fref(col[f]));
                    }
                    terms.push_back(cap_term(std::move(t)));
                    direct.push_back(0);
                } else {
                    terms.push_back({fref(r)});
                    direct.push_back(1);
                }
            }
        } else {
            std::vector<uint32_t> t;
            for (uint32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) t.push_back(fref(col[e]));
            terms.push_back(cap_term(std::move(t)));
            direct.push_back(0);
        }
        SN x;
        x.terms = std::move(terms);
        x.direct = std::move(direct);
        sn.push_back(std::move(x));
        sid[i] = static_cast<uint32_t>(sn.size() - 1);
    }
    if (bad) return P;
    const uint32_t M = static_cast<uint32_t>(sn.size());
    if (sid[root] == 0xFFFFFFFFu) return P;
    // ASAP levels (children come first in sn, since DAG children precede parents)
    std::vector<uint32_t> lev(M, 0);
    uint32_t Lmax = 0;
    for (uint32_t s = 0; s < M; ++s) {
        uint32_t l = 0;
        for (const auto &t : sn[s].terms)
            for (uint32_t r : t)
                if ((r >> 30) == TAG_NODE) {
                    if (r >= s) return P;
                    l = std::max(l, lev[r]);
                }
        lev[s] = l + 1;
        Lmax = std::max(Lmax, lev[s]);
    }
    const uint32_t sroot = sid[root];
    if (lev[sroot] != Lmax) return P;
    for (uint32_t s = 0; s < M; ++s)
        if (lev[s] == Lmax && s != sroot) return P;               // unreachable super-nodes
    std::vector<uint32_t> order(M), newid(M);
    for (uint32_t s = 0; s < M; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return lev[a] < lev[b]; });
    for (uint32_t j = 0; j < M; ++j) newid[order[j]] = j;
    auto pref = [&](uint32_t r) -> uint32_t {
        return (r >> 30) == TAG_NODE ? newid[r] : encode_leaf(r, var_field);
    };
    P.level_ptr.assign(Lmax + 1, 0);
    for (uint32_t s = 0; s < M; ++s) P.level_ptr[lev[s]]++;
    for (uint32_t l = 1; l <= Lmax; ++l) P.level_ptr[l] += P.level_ptr[l - 1];
    P.fptr.assign(M + 1, 0);
    // occurrences per target
    std::vector<uint32_t> selpos(n_sel, 0);
    for (uint32_t k = 0; k < n_sel; ++k) selpos[vsel[k]] = k;
    const size_t T = static_cast<size_t>(M) + n_ind + n_sel + n_angle_slots;
    std::vector<std::vector<std::array<uint32_t, 4>>> occ(T);
    for (uint32_t j = 0; j < M; ++j) {
        const SN &x = sn[order[j]];
        uint32_t nf = 0;
        for (size_t ti = 0; ti < x.terms.size(); ++ti) {
            const auto &t = x.terms[ti];
            for (size_t f = 0; f < t.size(); ++f) {
                P.frec.push_back(static_cast<uint64_t>(pref(t[f])) | (f + 1 == t.size() ? SOP_LAST_OF_TERM : 0ull) |
                                 (x.direct[ti] ? SOP_DIRECT : 0ull));
                ++nf;
                // occurrence of t[f] as a factor
                const uint32_t r = t[f], tag = r >> 30;
                int64_t tg = -1;
                if (tag == TAG_NODE) tg = newid[r];
                else if (tag == TAG_IND) {
                    const uint32_t xx = r & REF_MASK;
                    tg = static_cast<int64_t>(M) + ind_base[xx & 0xffffffu] + (xx >> 24);
                } else if (tag == TAG_SEL) {
                    tg = static_cast<int64_t>(M) + n_ind + selpos[r & REF_MASK];
                } else if (tag == TAG_SLOT && (r & REF_MASK) < n_angle_slots) {
                    tg = static_cast<int64_t>(M) + n_ind + n_sel + (r & REF_MASK);   // gradients in theta
                }
                if (tag == TAG_NODE) ++P.node_factors;
                if (tg < 0) continue;                             // other weights need no adjoint
                std::array<uint32_t, 4> rec = {j, NO_SIBLING, NO_SIBLING, NO_SIBLING};
                int k = 1;
                uint64_t reads = 1;                               // the parent's adjoint row
                for (size_t g = 0; g < t.size(); ++g)
                    if (g != f) {
                        reads += (t[g] >> 30) == TAG_NODE;
                        rec[k++] = pref(t[g]);
                    }
                if (tag == TAG_NODE) P.down_reads += reads;
                else if (tag != TAG_SLOT) P.leaf_reads += reads;
                occ[tg].push_back(rec);
            }
        }
        P.fptr[j + 1] = P.fptr[j] + nf;
        P.max_factors = std::max(P.max_factors, nf);
    }
    P.ostart.assign(T + 1, 0);
    for (size_t t = 0; t < T; ++t) {
        P.ostart[t + 1] = P.ostart[t] + static_cast<uint32_t>(occ[t].size());
        for (const auto &rec : occ[t]) P.occ.insert(P.occ.end(), rec.begin(), rec.end());
    }
    for (uint32_t k = 0; k < n_sel; ++k)
        P.osel.insert(P.osel.end(), occ[static_cast<size_t>(M) + n_ind + k].size(), vsel[k]);
    for (size_t t = 0; t < static_cast<size_t>(M) + n_ind + n_sel; ++t)
        for (const auto &rec : occ[t])
            for (uint32_t k = 1; k < 4; ++k)
                if (rec[k] != NO_SIBLING) P.max_sib = std::max(P.max_sib, k);
    // rows of the upward pass alone: super-node j lives from its level to the
    // level of its last consumer (the root to the end); rows are handed out
    // in level order and freed after their last reading level
    {
        std::vector<uint32_t> lvl(M), death(M, 0);
        for (uint32_t l = 0; l < Lmax; ++l)
            for (uint32_t j = P.level_ptr[l]; j < P.level_ptr[l + 1]; ++j) lvl[j] = l;
        for (uint32_t j = 0; j < M; ++j)
            for (uint32_t f = P.fptr[j]; f < P.fptr[j + 1]; ++f) {
                const uint32_t r = static_cast<uint32_t>(P.frec[f]);
                if ((r >> 30) == TAG_NODE) death[r] = std::max(death[r], lvl[j]);
            }
        death[P.root] = Lmax;
        std::vector<std::vector<uint32_t>> freed_after(Lmax + 1);
        std::vector<uint32_t> free_rows;
        P.srow.assign(M, 0);
        uint32_t next = 0;
        for (uint32_t l = 0; l < Lmax; ++l) {
            if (l > 0)                                   // rows whose last reader ran at level l - 1
                for (uint32_t r : freed_after[l - 1]) free_rows.push_back(r);
            for (uint32_t j = P.level_ptr[l]; j < P.level_ptr[l + 1]; ++j) {
                uint32_t r;
                if (!free_rows.empty()) {
                    r = free_rows.back();
                    free_rows.pop_back();
                } else {
                    r = next++;
                }
                P.srow[j] = r;
                freed_after[std::max(death[j], l)].push_back(r);
            }
        }
        P.live_rows = next;
        P.frec_live = P.frec;
        for (uint64_t &f : P.frec_live) {
            const uint32_t r = static_cast<uint32_t>(f);
            if ((r >> 30) == TAG_NODE) f = (f & ~0xffffffffull) | P.srow[r];
        }
    }
    P.S = M;
    P.L = Lmax;
    P.root = newid[sroot];
    P.ok = true;
    return P;
}

}  // namespace

extern "C" const char *ac_last_error(void) { return g_last_error.c_str(); }

extern "C" ac_status ac_load(const void *blob, size_t nbytes, int device, ac_graph **out) {
    if (!blob || !out) return fail(AC_ERR_INVALID_ARG, "ac_load: null blob or out pointer");
    *out = nullptr;
    Reader rd{static_cast<const uint8_t *>(blob), nbytes};
    const uint8_t *magic = rd.take_packed<uint8_t>(8);
    const uint32_t *h = rd.take_packed<uint32_t>(14);
    if (!rd.ok) return fail(AC_ERR_FORMAT, "ac_load: blob shorter than its header");
    if (std::memcmp(magic, MAGIC, 8) != 0) return fail(AC_ERR_FORMAT, "ac_load: bad magic");
    if (h[0] != 2) return fail(AC_ERR_FORMAT, "ac_load: unsupported version %u", h[0]);
    const uint32_t n_qubits = h[2], n_vars = h[3], n_words = h[4], n_angles = h[5], n_noise = h[6];
    const uint32_t n_slots = h[7], n_angle_slots = h[8], N = h[9], E = h[10], L = h[11], root = h[12];
    const uint32_t n_sel = h[13];
    if (n_qubits < 1 || n_vars < n_qubits || n_vars >= (1u << 20))
        return fail(AC_ERR_FORMAT, "ac_load: bad variable counts (%u qubits, %u vars)", n_qubits, n_vars);
    if (n_words < 1 || n_words > static_cast<uint32_t>(MAX_WORDS))
        return fail(AC_ERR_FORMAT, "ac_load: n_words %u outside [1, %d]", n_words, MAX_WORDS);
    if (n_angles > static_cast<uint32_t>(MAX_ANGLES)) return fail(AC_ERR_FORMAT, "ac_load: too many angles");
    if (n_angle_slots > n_slots || n_angle_slots > static_cast<uint32_t>(MAX_ANGLE_SLOTS))
        return fail(AC_ERR_FORMAT, "ac_load: bad angle-slot count %u", n_angle_slots);
    if (N < 1 || L < 1 || L > N || E < N || root >= N)
        return fail(AC_ERR_FORMAT, "ac_load: bad DAG sizes (N=%u E=%u L=%u root=%u)", N, E, L, root);
    if (N > REF_MASK || n_slots > REF_MASK || n_sel >= (MULTI_SIBLING & REF_MASK))
        return fail(AC_ERR_FORMAT, "ac_load: too many nodes, slots or selectors for 30-bit references");

    const uint8_t *var_dom = rd.take<uint8_t>(n_vars);
    const uint8_t *var_kind = rd.take_packed<uint8_t>(n_vars);
    const uint32_t *var_off = rd.take<uint32_t>(n_vars);
    const double *noise_def = rd.take<double>(n_noise);
    const SlotDesc *slots = rd.take_packed<SlotDesc>(n_slots);
    const uint32_t *selrec = rd.take_packed<uint32_t>(static_cast<size_t>(n_sel) * (1 + SEL_DOM));
    const uint8_t *op = rd.take_packed<uint8_t>(N);
    const uint32_t *row_ptr = rd.take<uint32_t>(N + 1);
    const uint32_t *col = rd.take<uint32_t>(E);
    const uint32_t *level_ptr = rd.take<uint32_t>(L + 1);
    if (!rd.ok) return fail(AC_ERR_FORMAT, "ac_load: blob truncated");

    // ---- evidence variables
    std::vector<uint32_t> ind_base(n_vars + 1, 0), var_field(n_vars);
    for (uint32_t v = 0; v < n_vars; ++v) {
        const uint32_t d = var_dom[v];
        if (d < 2 || d > static_cast<uint32_t>(MAX_DOM) || (d & (d - 1)) != 0)
            return fail(AC_ERR_FORMAT, "ac_load: variable %u domain %u (a power of two from 2 to %d)", v, d, MAX_DOM);
        if (var_kind[v] > 3) return fail(AC_ERR_FORMAT, "ac_load: variable %u kind %u", v, var_kind[v]);
        if ((v < n_qubits) != (var_kind[v] == 0)) return fail(AC_ERR_FORMAT, "ac_load: outputs must come first");
        uint32_t width = 0;
        while ((1u << width) < d) ++width;
        if (width > 4) return fail(AC_ERR_FORMAT, "ac_load: field too wide");
        const uint32_t word = var_off[v] / 64, shift = var_off[v] % 64;
        if (word >= n_words || shift + width > 64) return fail(AC_ERR_FORMAT, "ac_load: variable %u field out of range", v);
        var_field[v] = (word << 8) | (shift << 2) | (width - 1);
        ind_base[v + 1] = ind_base[v] + d;
    }
    const uint32_t n_ind = ind_base[n_vars];

    // ---- slots
    for (uint32_t s = 0; s < n_slots; ++s) {
        const SlotDesc &sd = slots[s];
        const bool angle = sd.base >= B_COS && sd.base <= B_EXPP;
        if (sd.base > B_SQRT_P || sd.coef > 3) return fail(AC_ERR_FORMAT, "ac_load: slot %u kind", s);
        if (angle != (s < n_angle_slots)) return fail(AC_ERR_FORMAT, "ac_load: angle slots must come first");
        if (angle && (sd.index < 0 || static_cast<uint32_t>(sd.index) >= n_angles || !std::isfinite(sd.scale)))
            return fail(AC_ERR_FORMAT, "ac_load: slot %u angle index %d", s, sd.index);
        if (sd.base >= B_SQRT_1MP && (sd.index < 0 || static_cast<uint32_t>(sd.index) >= n_noise))
            return fail(AC_ERR_FORMAT, "ac_load: slot %u noise index %d", s, sd.index);
        if (sd.base == B_CONST && (!std::isfinite(sd.re) || !std::isfinite(sd.im)))
            return fail(AC_ERR_FORMAT, "ac_load: slot %u constant not finite", s);
    }
    // ---- selectors: {variable, slot per value}; weights must not depend on theta
    std::vector<uint32_t> sel_dev(static_cast<size_t>(n_sel) * SEL_REC, 0), vsel_ptr(n_vars + 1, 0), vsel(n_sel);
    for (uint32_t q = 0; q < n_sel; ++q) {
        const uint32_t *r = selrec + static_cast<size_t>(q) * (1 + SEL_DOM);
        const uint32_t v = r[0];
        if (v >= n_vars || v < n_qubits || var_dom[v] > SEL_DOM)
            return fail(AC_ERR_FORMAT, "ac_load: selector %u variable %u", q, v);
        sel_dev[q * SEL_REC] = var_field[v];
        for (int u = 0; u < SEL_DOM; ++u) {
            const uint32_t sl = r[1 + u];
            if (sl != NO_SLOT && (sl >= n_slots || sl < n_angle_slots || u >= var_dom[v]))
                return fail(AC_ERR_FORMAT, "ac_load: selector %u slot %u", q, sl);
            sel_dev[q * SEL_REC + 1 + u] = sl;
        }
        vsel_ptr[v + 1]++;
    }
    for (uint32_t v = 0; v < n_vars; ++v) vsel_ptr[v + 1] += vsel_ptr[v];
    {
        std::vector<uint32_t> fs(vsel_ptr.begin(), vsel_ptr.end() - 1);
        for (uint32_t q = 0; q < n_sel; ++q) vsel[fs[selrec[static_cast<size_t>(q) * (1 + SEL_DOM)]]++] = q;
    }
    for (uint32_t m = 0; m < n_noise; ++m)
        if (!(noise_def[m] >= 0.0 && noise_def[m] <= 1.0)) return fail(AC_ERR_FORMAT, "ac_load: noise %u outside [0,1]", m);

    // ---- DAG
    if (row_ptr[0] != 0 || row_ptr[N] != E) return fail(AC_ERR_FORMAT, "ac_load: row_ptr ends");
    if (level_ptr[0] != 0 || level_ptr[L] != N) return fail(AC_ERR_FORMAT, "ac_load: level_ptr ends");
    for (uint32_t l = 0; l < L; ++l)                   // whole table first: strictly increasing up to N
        if (level_ptr[l + 1] <= level_ptr[l] || level_ptr[l + 1] > N)
            return fail(AC_ERR_FORMAT, "ac_load: empty or out-of-range level %u", l);
    std::vector<uint32_t> level(N);
    uint32_t max_width = 0;
    for (uint32_t l = 0; l < L; ++l) {
        max_width = std::max(max_width, level_ptr[l + 1] - level_ptr[l]);
        for (uint32_t i = level_ptr[l]; i < level_ptr[l + 1]; ++i) level[i] = l;
    }
    if (level[root] != L - 1 || level_ptr[L - 1] != N - 1)
        return fail(AC_ERR_FORMAT, "ac_load: the root must be the only node of the top level");
    std::vector<uint32_t> dcol(E), edge_parent(E);
    std::vector<uint32_t> n_par(N, 0), n_leafpar(n_ind + n_slots + n_sel, 0);
    int64_t flops = 0;
    for (uint32_t i = 0; i < N; ++i) {
        if (op[i] > 1) return fail(AC_ERR_FORMAT, "ac_load: node %u op %u", i, op[i]);
        if (row_ptr[i + 1] <= row_ptr[i]) return fail(AC_ERR_FORMAT, "ac_load: node %u has no children", i);
        const int64_t k = row_ptr[i + 1] - row_ptr[i];
        flops += (op[i] ? 6 : 2) * (k - 1);
        for (uint32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const uint32_t r = col[e], tag = r >> 30, x = r & REF_MASK;
            edge_parent[e] = i;
            if (tag == TAG_NODE) {
                if (x >= N || level[x] >= level[i]) return fail(AC_ERR_FORMAT, "ac_load: edge %u child %u not below node %u", e, x, i);
                n_par[x]++;
                dcol[e] = r;
            } else if (tag == TAG_IND) {
                const uint32_t v = x & 0xffffffu, u = x >> 24;
                if (v >= n_vars || u >= var_dom[v]) return fail(AC_ERR_FORMAT, "ac_load: edge %u indicator (%u,%u)", e, v, u);
                const uint32_t fld = var_field[v];
                dcol[e] = dev_ind_ref(u, (fld & 3u) + 1u, fld >> 8, (fld >> 2) & 63u);
                n_leafpar[ind_base[v] + u]++;
            } else if (tag == TAG_SLOT) {
                if (x >= n_slots) return fail(AC_ERR_FORMAT, "ac_load: edge %u slot %u", e, x);
                dcol[e] = r;
                n_leafpar[n_ind + x]++;
            } else {
                if (x >= n_sel) return fail(AC_ERR_FORMAT, "ac_load: edge %u selector %u", e, x);
                dcol[e] = r;
                n_leafpar[n_ind + n_slots + x]++;
            }
        }
    }
    // parent CSR of internal nodes and of leaves (edges in increasing order)
    const uint32_t n_leaves = n_ind + n_slots + n_sel;
    std::vector<uint32_t> par_ptr(N + 1, 0), leaf_ptr(n_leaves + 1, 0);
    for (uint32_t i = 0; i < N; ++i) par_ptr[i + 1] = par_ptr[i] + n_par[i];
    for (uint32_t i = 0; i < n_leaves; ++i) leaf_ptr[i + 1] = leaf_ptr[i] + n_leafpar[i];
    std::vector<uint32_t> par_edge(par_ptr[N]), leaf_edge(leaf_ptr[n_leaves]);
    {
        std::vector<uint32_t> fp(par_ptr.begin(), par_ptr.end() - 1), fl(leaf_ptr.begin(), leaf_ptr.end() - 1);
        for (uint32_t e = 0; e < E; ++e) {
            const uint32_t r = col[e], tag = r >> 30, x = r & REF_MASK;
            if (tag == TAG_NODE) par_edge[fp[x]++] = e;
            else if (tag == TAG_IND) leaf_edge[fl[ind_base[x & 0xffffffu] + (x >> 24)]++] = e;
            else if (tag == TAG_SLOT) leaf_edge[fl[n_ind + x]++] = e;
            else leaf_edge[fl[n_ind + n_slots + x]++] = e;
        }
    }

    // parent-edge records in the order of par_edge / leaf_edge: parent | sibling << 32,
    // the sibling being the other child of a two-child product (device
    // encoding), NO_SIBLING for a sum parent, MULTI_SIBLING for a product
    // with three or more children
    auto edge_record = [&](uint32_t e) -> uint64_t {
        const uint32_t p = edge_parent[e];
        const uint32_t r0 = row_ptr[p], r1 = row_ptr[p + 1];
        uint32_t sib = NO_SIBLING;
        if (op[p] != 0) sib = r1 - r0 == 2 ? dcol[e == r0 ? r0 + 1 : r0] : MULTI_SIBLING;
        return static_cast<uint64_t>(p) | (static_cast<uint64_t>(sib) << 32);
    };
    std::vector<uint64_t> par_rec(par_edge.size()), leaf_rec(leaf_edge.size());
    for (size_t q = 0; q < par_edge.size(); ++q) par_rec[q] = edge_record(par_edge[q]);
    for (size_t q = 0; q < leaf_edge.size(); ++q) leaf_rec[q] = edge_record(leaf_edge[q]);

    // ---- most-probable-explanation plan (MpePlan): the nodes with a noise-event
    // indicator below, and whether max-product over the events is exact here:
    // no selector leaves (they fold the events into weights), outputs at bits
    // 0..n-1, and every such sum node a decision on one evidence variable
    // (each branch an indicator of it, or a product with one, values distinct).
    // Decomposability over the events is the compiler's guarantee.
    std::vector<uint8_t> big(N, 0);
    std::vector<uint64_t> event_mask(n_words, 0);
    for (uint32_t v = n_qubits; v < n_vars; ++v) {
        const uint32_t fld = var_field[v], width = (fld & 3u) + 1u;
        event_mask[fld >> 8] |= ((1ull << width) - 1ull) << ((fld >> 2) & 63u);
    }
    std::string mpe_why;
    if (n_sel) mpe_why = "selector leaves fold the noise events into weights (compile with the events explicit)";
    for (uint32_t q = 0; q < n_qubits && mpe_why.empty(); ++q)
        if (var_off[q] != q) mpe_why = "outputs must occupy bits 0..n-1";
    auto direct_inds = [&](uint32_t r, std::vector<uint32_t> &out) {   // (var << 8 | value) of r's indicators
        out.clear();
        const uint32_t tag = r >> 30, x = r & REF_MASK;
        if (tag == TAG_IND) out.push_back(((x & 0xffffffu) << 8) | (x >> 24));
        else if (tag == TAG_NODE && op[x] == 1)
            for (uint32_t e = row_ptr[x]; e < row_ptr[x + 1]; ++e)
                if ((col[e] >> 30) == TAG_IND) out.push_back(((col[e] & 0xffffffu) << 8) | ((col[e] & REF_MASK) >> 24));
    };
    {
        std::vector<uint32_t> first, other;
        for (uint32_t i = 0; i < N; ++i) {
            for (uint32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
                const uint32_t r = col[e], tag = r >> 30, x = r & REF_MASK;
                if ((tag == TAG_NODE && big[x]) || (tag == TAG_IND && (x & 0xffffffu) >= n_qubits)) big[i] = 1;
            }
            if (!big[i] || op[i] != 0 || !mpe_why.empty()) continue;
            direct_inds(col[row_ptr[i]], first);
            bool decided = false;
            for (uint32_t cand : first) {
                const uint32_t v = cand >> 8;
                std::vector<uint32_t> seen;
                bool ok = true;
                for (uint32_t e = row_ptr[i]; e < row_ptr[i + 1] && ok; ++e) {
                    direct_inds(col[e], other);
                    uint32_t hits = 0, u = 0;
                    for (uint32_t o : other)
                        if ((o >> 8) == v) ++hits, u = o & 0xffu;
                    ok = hits == 1 && std::find(seen.begin(), seen.end(), u) == seen.end();
                    seen.push_back(u);
                }
                if (ok) {
                    decided = true;
                    break;
                }
            }
            if (!decided) {
                char buf[160];
                std::snprintf(buf, sizeof(buf), "sum node %u has a noise event below it but decides no single "
                              "variable (compile with the events decided first)", i);
                mpe_why = buf;
            }
        }
    }

    HostPlan hp = build_plan(N, op, row_ptr, col, root, ind_base, var_field, n_ind, n_sel, n_slots, sel_dev,
                             vsel_ptr, vsel);
    HostSop hs = build_sop(N, op, row_ptr, col, root, ind_base, var_field, n_ind, n_sel, vsel, n_angle_slots);

    // ---- device copy: one allocation, 256-byte aligned sections
    struct Sec { const void *src; size_t bytes; size_t off; };
    std::vector<Sec> secs = {
        {op, N * sizeof(uint8_t), 0},
        {row_ptr, (N + 1) * sizeof(uint32_t), 0},
        {dcol.data(), E * sizeof(uint32_t), 0},
        {level_ptr, (L + 1) * sizeof(uint32_t), 0},
        {slots, n_slots * sizeof(SlotDesc), 0},
        {par_ptr.data(), par_ptr.size() * sizeof(uint32_t), 0},
        {par_edge.data(), par_edge.size() * sizeof(uint32_t), 0},
        {edge_parent.data(), E * sizeof(uint32_t), 0},
        {leaf_ptr.data(), leaf_ptr.size() * sizeof(uint32_t), 0},
        {leaf_edge.data(), leaf_edge.size() * sizeof(uint32_t), 0},
        {var_field.data(), n_vars * sizeof(uint32_t), 0},
        {ind_base.data(), ind_base.size() * sizeof(uint32_t), 0},
        {noise_def, n_noise * sizeof(double), 0},
        {sel_dev.data(), sel_dev.size() * sizeof(uint32_t), 0},
        {vsel_ptr.data(), vsel_ptr.size() * sizeof(uint32_t), 0},
        {vsel.data(), vsel.size() * sizeof(uint32_t), 0},
        {hp.fwd.data(), hp.fwd.size() * sizeof(uint64_t), 0},
        {hp.level_ptr.data(), hp.level_ptr.size() * sizeof(uint32_t), 0},
        {hp.level_prod.data(), hp.level_prod.size() * sizeof(uint32_t), 0},
        {hp.brec.data(), hp.brec.size() * sizeof(uint32_t), 0},
        {hp.orec.data(), hp.orec.size() * sizeof(uint64_t), 0},
        {hp.estart.data(), hp.estart.size() * sizeof(uint32_t), 0},
        {hp.edg.data(), hp.edg.size() * sizeof(uint64_t), 0},
        {hp.fwd_u.data(), hp.fwd_u.size() * sizeof(uint64_t), 0},
        {hp.edg_u.data(), hp.edg_u.size() * sizeof(uint64_t), 0},
        {hp.dstart.data(), hp.dstart.size() * sizeof(uint32_t), 0},
        {hp.dterm.data(), hp.dterm.size() * sizeof(uint64_t), 0},
        {par_rec.data(), par_rec.size() * sizeof(uint64_t), 0},
        {leaf_rec.data(), leaf_rec.size() * sizeof(uint64_t), 0},
        {hp.esel.data(), hp.esel.size() * sizeof(uint32_t), 0},
        {hs.level_ptr.data(), hs.level_ptr.size() * sizeof(uint32_t), 0},
        {hs.fptr.data(), hs.fptr.size() * sizeof(uint32_t), 0},
        {hs.frec.data(), hs.frec.size() * sizeof(uint64_t), 0},
        {hs.ostart.data(), hs.ostart.size() * sizeof(uint32_t), 0},
        {hs.occ.data(), hs.occ.size() * sizeof(uint32_t), 0},
        {hs.osel.data(), hs.osel.size() * sizeof(uint32_t), 0},
        {hs.frec_live.data(), hs.frec_live.size() * sizeof(uint64_t), 0},
        {hs.srow.data(), hs.srow.size() * sizeof(uint32_t), 0},
        {big.data(), big.size() * sizeof(uint8_t), 0},
        {event_mask.data(), event_mask.size() * sizeof(uint64_t), 0},
    };
    size_t total = 0;
    for (auto &s : secs) {
        s.off = total;
        total += align256(std::max<size_t>(s.bytes, 1));
    }
    std::vector<uint8_t> host(total, 0);
    for (auto &s : secs)
        if (s.bytes) std::memcpy(host.data() + s.off, s.src, s.bytes);

    int n_dev = 0;
    hipError_t e = hipGetDeviceCount(&n_dev);
    if (e != hipSuccess || n_dev < 1) return fail(AC_ERR_DEVICE, "ac_load: no HIP device available");
    if (device < 0 || device >= n_dev) return fail(AC_ERR_INVALID_ARG, "ac_load: device %d of %d", device, n_dev);
    int prev = 0;
    (void)hipGetDevice(&prev);
    if ((e = hipSetDevice(device)) != hipSuccess) return fail_hip(e, "ac_load: hipSetDevice");
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) {
        (void)hipSetDevice(prev);
        return fail_hip(e, "ac_load: hipGetDeviceProperties");
    }
    if (device >= MAX_DEVICES) {
        (void)hipSetDevice(prev);
        return fail(AC_ERR_UNSUPPORTED, "ac_load: device index %d above %d", device, MAX_DEVICES - 1);
    }
    if ((e = resolve_scratch(device)) != hipSuccess) {
        (void)hipSetDevice(prev);
        return fail_hip(e, "ac_load: address of the static scratch");
    }
    void *dmem = nullptr;
    if ((e = hipMalloc(&dmem, total)) != hipSuccess) {
        (void)hipSetDevice(prev);
        return fail_hip(e, "ac_load: hipMalloc");
    }
    if ((e = hipMemcpy(dmem, host.data(), total, hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(dmem);
        (void)hipSetDevice(prev);
        return fail_hip(e, "ac_load: hipMemcpy");
    }
    (void)hipSetDevice(prev);

    ac_graph *g = new (std::nothrow) ac_graph();
    if (!g) {
        (void)hipFree(dmem);
        return fail(AC_ERR_OOM, "ac_load: host allocation");
    }
    auto at = [&](int k) { return static_cast<uint8_t *>(dmem) + secs[k].off; };
    DevGraph &d = g->dev;
    d.op = at(0);
    d.row_ptr = reinterpret_cast<const uint32_t *>(at(1));
    d.col = reinterpret_cast<const uint32_t *>(at(2));
    d.level_ptr = reinterpret_cast<const uint32_t *>(at(3));
    d.slots = reinterpret_cast<const SlotDesc *>(at(4));
    d.par_ptr = reinterpret_cast<const uint32_t *>(at(5));
    d.par_edge = reinterpret_cast<const uint32_t *>(at(6));
    d.edge_parent = reinterpret_cast<const uint32_t *>(at(7));
    d.leaf_ptr = reinterpret_cast<const uint32_t *>(at(8));
    d.leaf_edge = reinterpret_cast<const uint32_t *>(at(9));
    d.var_field = reinterpret_cast<const uint32_t *>(at(10));
    d.ind_base = reinterpret_cast<const uint32_t *>(at(11));
    d.noise_default = reinterpret_cast<const double *>(at(12));
    d.sel = reinterpret_cast<const uint32_t *>(at(13));
    d.vsel_ptr = reinterpret_cast<const uint32_t *>(at(14));
    d.vsel = reinterpret_cast<const uint32_t *>(at(15));
    d.par_rec = reinterpret_cast<const uint64_t *>(at(27));
    d.leaf_rec = reinterpret_cast<const uint64_t *>(at(28));
    d.n_sel = static_cast<int32_t>(n_sel);
    g->mpe.big = at(38);
    g->mpe.event_mask = reinterpret_cast<const uint64_t *>(at(39));
    g->mpe.n_qubits = static_cast<int32_t>(n_qubits);
    g->mpe_why = mpe_why;
    if (hp.ok) {
        LdsPlan &lp = g->plan;
        lp.fwd = reinterpret_cast<const uint64_t *>(at(16));
        lp.level_ptr = reinterpret_cast<const uint32_t *>(at(17));
        lp.level_prod = reinterpret_cast<const uint32_t *>(at(18));
        lp.brec = reinterpret_cast<const uint32_t *>(at(19));
        lp.orec = reinterpret_cast<const uint64_t *>(at(20));
        lp.estart = reinterpret_cast<const uint32_t *>(at(21));
        lp.edg = reinterpret_cast<const uint64_t *>(at(22));
        lp.fwd_u = reinterpret_cast<const uint64_t *>(at(23));
        lp.edg_u = reinterpret_cast<const uint64_t *>(at(24));
        lp.dstart = reinterpret_cast<const uint32_t *>(at(25));
        lp.dterm = reinterpret_cast<const uint64_t *>(at(26));
        lp.esel = reinterpret_cast<const uint32_t *>(at(29));
        lp.max_edges = static_cast<int32_t>(hp.max_edges);
        lp.N = static_cast<int32_t>(hp.N);
        lp.L = static_cast<int32_t>(hp.L);
        lp.root = static_cast<int32_t>(hp.root);
        lp.R = static_cast<int64_t>(hp.orec.size());
        g->has_plan = true;
        g->plan_level_ptr = hp.level_ptr;
    }
    if (hs.ok) {
        SopPlan &sp = g->sop;
        sp.level_ptr = reinterpret_cast<const uint32_t *>(at(30));
        sp.fptr = reinterpret_cast<const uint32_t *>(at(31));
        sp.frec = reinterpret_cast<const uint64_t *>(at(32));
        sp.ostart = reinterpret_cast<const uint32_t *>(at(33));
        sp.occ = reinterpret_cast<const uint32_t *>(at(34));
        sp.osel = reinterpret_cast<const uint32_t *>(at(35));
        sp.S = static_cast<int32_t>(hs.S);
        sp.L = static_cast<int32_t>(hs.L);
        sp.root = static_cast<int32_t>(hs.root);
        sp.max_factors = static_cast<int32_t>(hs.max_factors);
        sp.frec_live = reinterpret_cast<const uint64_t *>(at(36));
        sp.srow = reinterpret_cast<const uint32_t *>(at(37));
        sp.live_rows = static_cast<int32_t>(hs.live_rows);
        // QKC_SAMPLE_SIB3=1 keeps the three-sibling groups on any plan (tests)
        const char *sib_env = std::getenv("QKC_SAMPLE_SIB3");
        sp.occ_sib3 = hs.max_sib > 2 || (sib_env && std::atoi(sib_env) == 1) ? 1 : 0;
        // the sampler's decision pass keeps one change bit per variable and
        // handles variables of at most SEL_DOM values
        bool small_doms = true;
        for (uint32_t v = 0; v < n_vars; ++v) small_doms = small_doms && var_dom[v] <= SEL_DOM;
        sp.mask_words = small_doms && n_vars <= 64u * MAX_MASK_WORDS ? static_cast<int32_t>((n_vars + 63) / 64) : 0;
        g->has_sop = true;
    }
    d.N = static_cast<int32_t>(N);
    d.E = E;
    d.L = static_cast<int32_t>(L);
    d.root = static_cast<int32_t>(root);
    d.S = static_cast<int32_t>(n_slots);
    d.S_ang = static_cast<int32_t>(n_angle_slots);
    d.n_vars = static_cast<int32_t>(n_vars);
    d.W = static_cast<int32_t>(n_words);
    d.n_ind = static_cast<int32_t>(n_ind);
    d.K = static_cast<int32_t>(n_angles);
    d.n_noise = static_cast<int32_t>(n_noise);
    d.n_qubits = static_cast<int32_t>(n_qubits);
    g->dmem = dmem;
    g->device = device;
    g->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    if (const char *env = std::getenv("QKC_STREAM_WAVES")) {
        const int nw = std::atoi(env);
        if (nw >= 1 && nw <= MAX_BLOCK / WAVE) g->stream_waves = nw;
    }
    if (const char *env = std::getenv("QKC_TILE_WAVES")) {
        const int nw = std::atoi(env);
        if (nw == 4 || nw == 8 || nw == 16) g->tile_waves = nw;
    }
    for (int k = 0; k < 4; ++k) {
        const int blk = k == 3 && g->stream_waves ? g->stream_waves * WAVE : BLOCK;
        g->resident[AC_C64][k] = resident_blocks<float>(d, g->sop, k, blk);
        g->resident[AC_C128][k] = resident_blocks<double>(d, g->sop, k, blk);
    }
    for (int k : {0, 1, 3})
        for (int j = 0; j < 3; ++j) {
            g->wide_resident[AC_C64][k][j] = resident_blocks<float>(d, g->sop, k, BLOCK << j);
            g->wide_resident[AC_C128][k][j] = resident_blocks<double>(d, g->sop, k, BLOCK << j);
        }
    g->var_dom.assign(var_dom, var_dom + n_vars);
    g->var_offset.assign(var_off, var_off + n_vars);
    ac_info_t &inf = g->info;
    inf.n_qubits = d.n_qubits;
    inf.n_vars = d.n_vars;
    inf.n_words = d.W;
    inf.n_angles = d.K;
    inf.n_noise = d.n_noise;
    inf.n_slots = d.S;
    inf.n_angle_slots = d.S_ang;
    inf.n_internal = d.N;
    inf.n_edges = d.E;
    inf.n_levels = d.L;
    inf.max_level_width = static_cast<int32_t>(max_width);
    inf.n_indicator_leaves = d.n_ind;
    inf.n_selectors = d.n_sel;
    inf.root = d.root;
    inf.device = device;
    inf.n_prod_flops = flops;
    inf.max_live = d.N;
    if (hs.ok) {
        inf.n_super = static_cast<int32_t>(hs.S);
        inf.n_super_levels = static_cast<int32_t>(hs.L);
        inf.n_super_node_factors = static_cast<int64_t>(hs.node_factors);
        inf.n_super_down_reads = static_cast<int64_t>(hs.down_reads);
        inf.n_super_leaf_reads = static_cast<int64_t>(hs.leaf_reads);
        inf.max_live = static_cast<int32_t>(hs.live_rows);
        inf.max_siblings = static_cast<int32_t>(hs.max_sib);
    }
    *out = g;
    return AC_OK;
}

extern "C" ac_status ac_free(ac_graph *g) {
    if (!g) return AC_OK;
    if (g->dmem) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(g->device);
        (void)hipFree(g->dmem);
        (void)hipSetDevice(prev);
    }
    delete g;
    return AC_OK;
}

extern "C" ac_status ac_info(const ac_graph *g, ac_info_t *info) {
    if (!g || !info) return fail(AC_ERR_INVALID_ARG, "ac_info: null argument");
    *info = g->info;
    return AC_OK;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------

namespace {

constexpr size_t WS_CAP = static_cast<size_t>(96) << 30;   // cap on per-call tile buffers (HBM is 288 GB)
constexpr size_t LDS_LIMIT = 64 * 1024;                     // dynamic LDS per workgroup

constexpr size_t CU_LDS = 160 * 1024;                      // LDS per compute unit (gfx950)

// Sampler kernels: the batched streaming kernel on the binary plan, the
// LDS-resident node-parallel kernel, or the plain streaming kernel on the
// blob's own DAG (used when no plan exists).  The streaming kernel has the
// higher throughput once the batch fills the chip; the LDS-resident one has a
// much shorter time per chain (its node values never leave the CU), so it
// wins for batches up to about ten times the number of chains it holds at
// once (complex64, 10 sweeps, noisy QAOA ACs of 937 to 3577 nodes, both
// kernels with their per-call workgroup shapes: the LDS kernel is faster at
// 8 such groups on every AC, slower at 16 on all but one where the two tie,
// and slower at 10.7 on the smallest).
// QKC_SAMPLE_KERNEL = stream | lds | global forces one (comparisons, tests);
// QKC_LDS_BATCH_FACTOR replaces the factor below (measurements).
enum SampleKernel { SK_STREAM, SK_LDS, SK_GLOBAL };

constexpr int64_t LDS_BATCH_FACTOR = 10;  // LDS kernel up to this many groups of resident chains

bool lds_capacity(const ac_graph *g, ac_dtype dt, int &cpw, int64_t &per_cu);

SampleKernel sample_kernel(const ac_graph *g, ac_dtype dt, int64_t chains) {
    // the streaming sampler runs on the sum-of-products plan and addresses a
    // workgroup's rows through a buffer resource with 32-bit offsets: its
    // region must stay below 2 GiB
    const size_t stream_rows = 2 * static_cast<size_t>(g->sop.S) + g->dev.n_ind;
    const bool stream_ok = g->has_sop && stream_rows * WAVE * (dt == AC_C64 ? 8 : 16) < (size_t{1} << 31);
    if (!g->has_plan) return stream_ok ? SK_STREAM : SK_GLOBAL;
    const char *kern = std::getenv("QKC_SAMPLE_KERNEL");
    if (kern && std::strcmp(kern, "global") == 0) return SK_GLOBAL;
    if (kern && std::strcmp(kern, "lds") == 0) return SK_LDS;
    if (kern && std::strcmp(kern, "stream") == 0) return stream_ok ? SK_STREAM : SK_GLOBAL;
    int cpw = 0;
    int64_t per_cu = 0;
    int64_t factor = LDS_BATCH_FACTOR;
    if (const char *env = std::getenv("QKC_LDS_BATCH_FACTOR")) factor = std::max(0, std::min(1 << 20, std::atoi(env)));
    if (lds_capacity(g, dt, cpw, per_cu) && chains <= factor * per_cu * cpw * static_cast<int64_t>(g->n_cu))
        return SK_LDS;
    return stream_ok ? SK_STREAM : SK_GLOBAL;
}

// Chains per wave and workgroups per CU of the LDS-resident sampler, or false
// if one chain's state does not fit in a CU's LDS.
bool lds_capacity(const ac_graph *g, ac_dtype dt, int &cpw, int64_t &per_cu) {
    if (!g->has_plan) return false;
    const size_t cb = dt == AC_C64 ? sample_lds_chain_bytes<float>(g->dev, g->plan)
                                   : sample_lds_chain_bytes<double>(g->dev, g->plan);
    const size_t meta = sample_lds_meta_bytes(g->plan);
    if (cb + meta > CU_LDS) return false;
    // chains per wave: minimise level steps per chain at the occupancy the LDS allows
    double best = -1.0;
    int best_cpw = 1;
    const char *env = std::getenv("QKC_SAMPLE_CPW");
    const int forced = env ? std::atoi(env) : 0;
    for (int c : {1, 2, 4}) {
        if (cb * c + meta > CU_LDS) continue;
        const int lpc = WAVE / c;
        double steps = 0;
        const auto &lvl = g->plan_level_ptr;
        for (size_t l = 1; l < lvl.size(); ++l) steps += static_cast<double>((lvl[l] - lvl[l - 1] + lpc - 1) / lpc);
        steps = 2.0 * steps + static_cast<double>((g->dev.n_ind + lpc - 1) / lpc);
        const double waves = static_cast<double>(CU_LDS / (cb * c + meta));
        const double rate = std::min(waves, 8.0) * c / steps;
        if (rate > best) {
            best = rate;
            best_cpw = c;
        }
        if (forced == c) {
            best = 1e300;
            best_cpw = c;
        }
    }
    cpw = best_cpw;
    per_cu = static_cast<int64_t>(CU_LDS / (cb * cpw + meta));
    return true;
}

// Waves per chain of the LDS-resident sampler: four when each wave holds one
// chain and at most five chains fit in a CU (a CU would otherwise run at most
// one or two waves per SIMD; five 4-wave workgroups is what its registers
// hold), else one.  Measured on noisy QAOA ACs of 1277 to 3577 nodes, 256 to
// 4096 chains: four waves 1.2-1.5x faster.  QKC_SAMPLE_WPC = 1 | 4 forces it.
int sample_lds_waves(const ac_graph *g, ac_dtype dt) {
    int cpw = 0;
    int64_t per_cu = 0;
    if (!lds_capacity(g, dt, cpw, per_cu)) return 1;
    if (const char *env = std::getenv("QKC_SAMPLE_WPC")) {
        const int w = std::atoi(env);
        if (w == 1 || (w == 4 && cpw == 1)) return w;
    }
    return cpw == 1 && per_cu <= 5 ? 4 : 1;
}

bool sample_lds_shape(const ac_graph *g, ac_dtype dt, int64_t chains, int &cpw, int &grid) {
    int64_t per_cu = 0;
    if (!lds_capacity(g, dt, cpw, per_cu)) return false;
    const int64_t want = (chains + cpw - 1) / cpw;
    grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, per_cu * g->n_cu)));
    return true;
}

// Threads per workgroup of a tile kernel (kid 0 upward pass, 1 gradients, 3
// streaming sampler) for a batch of `batch` elements or chains: 4, 8 or 16
// waves per 64-element tile, whichever keeps the most waves resident at once
// (ties: the smaller workgroup).  Full batches keep four waves; a small batch
// on a large AC gets its tiles' levels split over more waves instead of
// being held to one tile's level chain while most of the chip idles
// (measured on noisy QAOA ACs of 3.6k and 138k nodes, batches of 1306 to
// 262,144: the rule picked the fastest size at every point).
// QKC_STREAM_WAVES forces the sampler's size, QKC_TILE_WAVES (4, 8, 16) the
// others' and the max-product kernel's (measurements, tests).
int wide_block_for(const ac_graph *g, ac_dtype dt, int64_t batch, int kid, int &wg_per_cu) {
    if (kid == 3 && g->stream_waves) {
        wg_per_cu = g->resident[dt][3];
        return g->stream_waves * WAVE;
    }
    if (kid != 3 && g->tile_waves) {
        const int j = g->tile_waves == 4 ? 0 : g->tile_waves == 8 ? 1 : 2;
        wg_per_cu = std::max(1, g->wide_resident[dt][kid][j]);
        return BLOCK << j;
    }
    const int64_t tiles = std::max<int64_t>(1, (batch + WAVE - 1) / WAVE);
    int j = 0;
    int64_t best = -1;
    for (int jj = 0; jj < 3; ++jj) {      // most waves resident at once; ties go to smaller workgroups
        const int64_t wgs = std::min<int64_t>(tiles, static_cast<int64_t>(g->n_cu) * g->wide_resident[dt][kid][jj]);
        const int64_t waves = wgs * (4 << jj);
        if (waves > best) {
            best = waves;
            j = jj;
        }
    }
    wg_per_cu = std::max(1, g->wide_resident[dt][kid][j]);
    return BLOCK << j;
}

// The upward pass runs on the sum-of-products plan when there is one (rows
// only for super-nodes), else on the DAG.
SopPlan eval_plan(const ac_graph *g) { return g->has_sop ? g->sop : SopPlan{}; }
size_t eval_rows(const ac_graph *g) { return g->has_sop ? static_cast<size_t>(g->sop.S) : static_cast<size_t>(g->dev.N); }
// rows of the upward pass alone (super-node rows reused once their readers ran)
size_t eval_live_rows(const ac_graph *g) {
    return g->has_sop ? static_cast<size_t>(g->sop.live_rows) : static_cast<size_t>(g->dev.N);
}

struct Layout {
    size_t wfix_off = 0, contrib_off = 0, sort_off = 0, sort_bytes = 0, tiles_off = 0, total = 0;
    size_t per_wg_elems = 0;   // complex elements per workgroup buffer
    size_t cs = 8;             // bytes per complex element
    int grid = 0;
    int block = BLOCK;         // threads per workgroup
};

// The max-product kernel (a query over small ACs; complex128 rows) spreads
// each tile's levels over 16 waves, two such workgroups per CU (its register
// budget is bounded for 8 waves per SIMD).  Measured on 16-outcome queries
// of a 17k-node AC: 512 tiles 5.1 ms against 10.1 ms as four workgroups of
// 4 waves per CU and 6.3 ms as one of 16.
constexpr int MPE_WG_PER_CU = 2;

bool make_layout(const ac_graph *g, ac_dtype dt, int64_t batch, int op, Layout &out, size_t tile_cap = 0) {
    if (!g || batch < 0 || (dt != AC_C64 && dt != AC_C128) || op < 0 || op > 3) return false;
    if (op == AC_OP_MPE && dt != AC_C128) return false;
    const DevGraph &d = g->dev;
    const size_t cs = dt == AC_C64 ? 8 : 16;
    size_t rows = 0;
    int kid = 0;
    if (op == AC_OP_EVAL) rows = eval_live_rows(g);
    else if (op == AC_OP_MPE) rows = static_cast<size_t>(d.N);
    else if (op == AC_OP_GRAD) {
        rows = 2 * eval_rows(g) + d.S_ang + d.n_ind;
        kid = 1;
    } else {
        int cpw = 0, lgrid = 0;
        const SampleKernel sk = sample_kernel(g, dt, batch);
        if (sk == SK_LDS && sample_lds_shape(g, dt, batch, cpw, lgrid)) rows = 0;
        else if (sk == SK_STREAM) {
            rows = 2 * static_cast<size_t>(g->sop.S) + d.n_ind;
            kid = 3;
        } else {
            rows = 2 * static_cast<size_t>(d.N) + d.n_ind;
            kid = 2;
        }
    }
    const size_t per_wg = rows * WAVE;
    int64_t tiles = (batch + WAVE - 1) / WAVE;
    // persistent grids: exactly the workgroups that are resident together
    int wg_per_cu = g->resident[dt][kid];
    int block = BLOCK;
    if (op == AC_OP_MPE) {
        // fewer tiles than two per CU: each tile's levels spread over 16 waves
        wg_per_cu = MPE_WG_PER_CU;
        block = g->tile_waves ? g->tile_waves * WAVE : MAX_BLOCK;
    } else if (kid != 2) {
        block = wide_block_for(g, dt, batch, kid, wg_per_cu);
    }
    if (const char *env = std::getenv("QKC_WG_PER_CU")) wg_per_cu = std::max(1, std::min(16, std::atoi(env)));
    int64_t grid = std::min<int64_t>(tiles, static_cast<int64_t>(g->n_cu) * wg_per_cu);
    if (per_wg > 0) {
        size_t ws_cap = WS_CAP;
        if (const char *env = std::getenv("QKC_WS_CAP_GIB")) {
            const long v = std::atol(env);
            if (v >= 1 && v <= 256) ws_cap = static_cast<size_t>(v) << 30;
        }
        if (tile_cap) ws_cap = tile_cap;   // a fixed region (the static scratch)
        const int64_t cap = std::max<int64_t>(1, static_cast<int64_t>(ws_cap / (per_wg * cs)));
        grid = std::min(grid, cap);
    }
    if (batch > 0 && grid < 1) grid = 1;
    Layout L;
    size_t off = 0;
    L.wfix_off = off;                                    // fixed weights, 16 bytes each for both dtypes
    off += align256(static_cast<size_t>(std::max(d.S, 1)) * 16);
    L.contrib_off = off;
    if (op == AC_OP_GRAD) off += align256(static_cast<size_t>(std::max<int64_t>(batch, 1)) * std::max(d.K, 1) * 8);
    L.sort_off = off;
    if (op == AC_OP_GRAD) {
        L.sort_bytes = grad_sort_bytes(batch);
        off += align256(L.sort_bytes);
    }
    L.tiles_off = off;
    off += align256(static_cast<size_t>(grid) * per_wg * cs);
    L.total = off;
    L.per_wg_elems = per_wg;
    L.cs = cs;
    L.grid = static_cast<int>(grid);
    L.block = block;
    out = L;
    return true;
}

// A caller's workspace below the full layout: the grid shrinks to the
// per-workgroup regions that fit after the fixed part (at least one), so the
// call keeps fewer workgroups resident and leaves the rest of the device to
// other streams.  False if not even one region fits.
bool fit_workspace(Layout &L, size_t ws_bytes) {
    if (ws_bytes >= L.total) return true;
    const size_t per = L.per_wg_elems * L.cs;
    if (per == 0 || L.grid < 1 || ws_bytes < L.tiles_off + per) return false;
    const int64_t grid = static_cast<int64_t>((ws_bytes - L.tiles_off) / per);
    L.grid = static_cast<int>(std::min<int64_t>(L.grid, grid));
    L.total = L.tiles_off + static_cast<size_t>(L.grid) * per;
    return true;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

ac_status check_common(const ac_graph *g, ac_dtype dt, const double *theta, int32_t P, const char *who) {
    if (!g) return fail(AC_ERR_INVALID_ARG, "%s: null graph", who);
    if (dt != AC_C64 && dt != AC_C128) return fail(AC_ERR_INVALID_ARG, "%s: bad dtype %d", who, static_cast<int>(dt));
    if (P < 0) return fail(AC_ERR_INVALID_ARG, "%s: P < 0", who);
    if (g->dev.K > 0 && P > 0 && !theta) return fail(AC_ERR_INVALID_ARG, "%s: theta is null", who);
    return AC_OK;
}

}  // namespace

extern "C" size_t ac_workspace_size(const ac_graph *g, ac_dtype dtype, int64_t batch, int op) {
    Layout L;
    if (!make_layout(g, dtype, batch, op, L)) {
        fail(AC_ERR_INVALID_ARG, "ac_workspace_size: invalid arguments");
        return 0;
    }
    return L.total;
}

extern "C" size_t ac_workspace_size_share(const ac_graph *g, ac_dtype dtype, int64_t batch, int op, double share) {
    Layout L;
    if (!(share > 0.0 && share <= 1.0) || !make_layout(g, dtype, batch, op, L)) {
        fail(AC_ERR_INVALID_ARG, "ac_workspace_size_share: invalid arguments");
        return 0;
    }
    const size_t per = L.per_wg_elems * L.cs;
    if (per == 0 || L.grid <= 1) return L.total;
    const int64_t grid = std::max<int64_t>(1, static_cast<int64_t>(std::ceil(share * L.grid)));
    if (grid >= L.grid) return L.total;
    return L.tiles_off + static_cast<size_t>(grid) * per;
}

extern "C" ac_status ac_sample_shape(const ac_graph *g, ac_dtype dtype, int64_t chains, int32_t *kind,
                                     int64_t *concurrent) {
    if (!g || !kind || !concurrent || (dtype != AC_C64 && dtype != AC_C128) || chains < 1)
        return fail(AC_ERR_INVALID_ARG, "ac_sample_shape: invalid arguments");
    const SampleKernel sk = sample_kernel(g, dtype, chains);
    int cpw = 0, lgrid = 0;
    if (sk == SK_LDS && sample_lds_shape(g, dtype, chains, cpw, lgrid)) {
        int64_t per_cu = 0;
        lds_capacity(g, dtype, cpw, per_cu);
        *kind = AC_SAMPLER_LDS;
        *concurrent = std::min<int64_t>(chains, per_cu * cpw * static_cast<int64_t>(g->n_cu));
        return AC_OK;
    }
    Layout L;
    if (!make_layout(g, dtype, chains, AC_OP_SAMPLE, L)) return fail(AC_ERR_INVALID_ARG, "ac_sample_shape: no layout");
    *kind = sk == SK_STREAM ? AC_SAMPLER_STREAM : AC_SAMPLER_GLOBAL;
    *concurrent = std::min<int64_t>(chains, static_cast<int64_t>(L.grid) * WAVE);
    return AC_OK;
}

extern "C" ac_status ac_eval_batch(const ac_graph *g, ac_dtype dtype, const double *theta, int32_t P,
                                   const double *noise, const int32_t *param_of, const uint64_t *evidence,
                                   int64_t B, void *amp_out, double *prob_out, void *ws, size_t ws_bytes,
                                   void *stream) {
    ac_status s = check_common(g, dtype, theta, P, "ac_eval_batch");
    if (s != AC_OK) return s;
    if (lds_bytes(g->dev) > LDS_LIMIT)
        return fail(AC_ERR_UNSUPPORTED, "ac_eval_batch: evidence and angle tables exceed LDS");
    if (B < 0) return fail(AC_ERR_INVALID_ARG, "ac_eval_batch: B < 0");
    if (B == 0) return AC_OK;
    if (P < 1) return fail(AC_ERR_INVALID_ARG, "ac_eval_batch: P must be >= 1 when B > 0");
    if (!param_of || !evidence || !amp_out) return fail(AC_ERR_INVALID_ARG, "ac_eval_batch: null param_of/evidence/amp_out");
    Layout L;
    make_layout(g, dtype, B, AC_OP_EVAL, L);
    if (!ws || !fit_workspace(L, ws_bytes))
        return fail(AC_ERR_INVALID_ARG, "ac_eval_batch: workspace of %zu bytes, need %zu (%zu for one workgroup)",
                    ws_bytes, L.total, L.tiles_off + L.per_wg_elems * L.cs);
    DeviceGuard dg(g->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *w = static_cast<uint8_t *>(ws);
    hipError_t e;
    if (dtype == AC_C64) {
        e = launch_fixed_slots<float>(g->dev, noise, w + L.wfix_off, st);
        if (e == hipSuccess)
            e = launch_eval<float>(g->dev, eval_plan(g), L.grid, L.block, theta, param_of, P, evidence, B, w + L.wfix_off, w + L.tiles_off,
                                   L.per_wg_elems, amp_out, prob_out, st);
    } else {
        e = launch_fixed_slots<double>(g->dev, noise, w + L.wfix_off, st);
        if (e == hipSuccess)
            e = launch_eval<double>(g->dev, eval_plan(g), L.grid, L.block, theta, param_of, P, evidence, B, w + L.wfix_off, w + L.tiles_off,
                                    L.per_wg_elems, amp_out, prob_out, st);
    }
    if (e != hipSuccess) return fail_hip(e, "ac_eval_batch: launch");
    return AC_OK;
}

extern "C" ac_status ac_eval_batch_static(const ac_graph *g, ac_dtype dtype, const double *theta, int32_t P,
                                          const double *noise, const int32_t *param_of, const uint64_t *evidence,
                                          int64_t B, void *amp_out, double *prob_out, void *stream) {
    ac_status s = check_common(g, dtype, theta, P, "ac_eval_batch_static");
    if (s != AC_OK) return s;
    if (lds_bytes(g->dev) > LDS_LIMIT)
        return fail(AC_ERR_UNSUPPORTED, "ac_eval_batch_static: evidence and angle tables exceed LDS");
    if (B < 0) return fail(AC_ERR_INVALID_ARG, "ac_eval_batch_static: B < 0");
    if (B == 0) return AC_OK;
    if (P < 1) return fail(AC_ERR_INVALID_ARG, "ac_eval_batch_static: P must be >= 1 when B > 0");
    if (!param_of || !evidence || !amp_out)
        return fail(AC_ERR_INVALID_ARG, "ac_eval_batch_static: null param_of/evidence/amp_out");
    // the fixed weights come first; the rest of the scratch holds as many
    // workgroups' node rows as fit (the grid is capped to that number)
    const size_t cs = dtype == AC_C64 ? 8 : 16;
    const size_t wfix_bytes = align256(static_cast<size_t>(std::max(g->dev.S, 1)) * 16);
    const size_t one_tile = align256(eval_live_rows(g) * WAVE * cs);
    if (wfix_bytes + one_tile > STATIC_SCRATCH_BYTES)
        return fail(AC_ERR_UNSUPPORTED,
                    "ac_eval_batch_static: one 64-element tile needs %zu bytes of scratch (%zu node rows), above the "
                    "%zu-byte static scratch; use ac_eval_batch with a workspace",
                    wfix_bytes + one_tile, eval_live_rows(g), STATIC_SCRATCH_BYTES);
    Layout L;
    make_layout(g, dtype, B, AC_OP_EVAL, L, STATIC_SCRATCH_BYTES - wfix_bytes);
    if (L.total > STATIC_SCRATCH_BYTES)
        return fail(AC_ERR_UNSUPPORTED, "ac_eval_batch_static: layout of %zu bytes exceeds the static scratch", L.total);
    uint8_t *w = static_cast<uint8_t *>(scratch_of(g->device));
    if (!w) return fail(AC_ERR_DEVICE, "ac_eval_batch_static: static scratch of device %d not resolved", g->device);
    DeviceGuard dg(g->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (dtype == AC_C64) {
        e = launch_fixed_slots<float>(g->dev, noise, w + L.wfix_off, st);
        if (e == hipSuccess)
            e = launch_eval<float>(g->dev, eval_plan(g), L.grid, L.block, theta, param_of, P, evidence, B, w + L.wfix_off, w + L.tiles_off,
                                   L.per_wg_elems, amp_out, prob_out, st);
    } else {
        e = launch_fixed_slots<double>(g->dev, noise, w + L.wfix_off, st);
        if (e == hipSuccess)
            e = launch_eval<double>(g->dev, eval_plan(g), L.grid, L.block, theta, param_of, P, evidence, B, w + L.wfix_off, w + L.tiles_off,
                                    L.per_wg_elems, amp_out, prob_out, st);
    }
    if (e != hipSuccess) return fail_hip(e, "ac_eval_batch_static: launch");
    return AC_OK;
}

extern "C" ac_status ac_grad_batch(const ac_graph *g, ac_dtype dtype, const double *theta, int32_t P,
                                   const double *noise, const int32_t *param_of, const uint64_t *evidence,
                                   int64_t B, int mode, const void *cotangent, const double *weight,
                                   double *grad_theta, void *amp_out, void *dfdtheta_out, void *dind_out,
                                   void *ws, size_t ws_bytes, void *stream) {
    ac_status s = check_common(g, dtype, theta, P, "ac_grad_batch");
    if (s != AC_OK) return s;
    if (lds_bytes(g->dev) > LDS_LIMIT)
        return fail(AC_ERR_UNSUPPORTED, "ac_grad_batch: evidence and angle tables exceed LDS");
    if (B < 0) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: B < 0");
    if (mode < 0 || mode > 2) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: bad mode %d", mode);
    if (mode == AC_GRAD_COTANGENT && B > 0 && !cotangent) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: cotangent is null");
    if (mode != AC_GRAD_COTANGENT && B > 0 && !weight) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: weight is null");
    if (g->dev.K > 0 && P > 0 && !grad_theta) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: grad_theta is null");
    if (B > 0 && (!param_of || !evidence)) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: null param_of/evidence");
    if (B > 0 && P < 1) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: P must be >= 1 when B > 0");
    if (B > 0x7fffffff) return fail(AC_ERR_UNSUPPORTED, "ac_grad_batch: B above 2^31 - 1");
    Layout L;
    make_layout(g, dtype, B, AC_OP_GRAD, L);
    DeviceGuard dg(g->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (B == 0) {
        if (g->dev.K > 0 && P > 0) {
            hipError_t e = launch_zero_f64(grad_theta, static_cast<int64_t>(P) * g->dev.K, st);
            if (e != hipSuccess) return fail_hip(e, "ac_grad_batch: clear");
        }
        return AC_OK;
    }
    if (!ws || !fit_workspace(L, ws_bytes))
        return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: workspace of %zu bytes, need %zu (%zu for one workgroup)",
                    ws_bytes, L.total, L.tiles_off + L.per_wg_elems * L.cs);
    uint8_t *w = static_cast<uint8_t *>(ws);
    double *contrib = reinterpret_cast<double *>(w + L.contrib_off);
    hipError_t e;
    if (dtype == AC_C64) {
        e = launch_fixed_slots<float>(g->dev, noise, w + L.wfix_off, st);
        if (e == hipSuccess)
            e = launch_grad<float>(g->dev, eval_plan(g), L.grid, L.block, theta, param_of, evidence, B, w + L.wfix_off, w + L.tiles_off,
                                   L.per_wg_elems, mode, cotangent, weight, contrib, P, grad_theta, amp_out,
                                   dfdtheta_out, dind_out, w + L.sort_off, L.sort_bytes, st);
    } else {
        e = launch_fixed_slots<double>(g->dev, noise, w + L.wfix_off, st);
        if (e == hipSuccess)
            e = launch_grad<double>(g->dev, eval_plan(g), L.grid, L.block, theta, param_of, evidence, B, w + L.wfix_off, w + L.tiles_off,
                                    L.per_wg_elems, mode, cotangent, weight, contrib, P, grad_theta, amp_out,
                                    dfdtheta_out, dind_out, w + L.sort_off, L.sort_bytes, st);
    }
    if (e != hipSuccess) return fail_hip(e, "ac_grad_batch: launch");
    return AC_OK;
}

extern "C" ac_status ac_mpe_batch(const ac_graph *g, const double *theta, int32_t P, const double *noise,
                                  const int32_t *param_of, const uint64_t *evidence, int64_t B, double *prob_out,
                                  uint64_t *mpe_out, void *ws, size_t ws_bytes, void *stream) {
    ac_status s = check_common(g, AC_C128, theta, P, "ac_mpe_batch");
    if (s != AC_OK) return s;
    if (!g->mpe_why.empty()) return fail(AC_ERR_UNSUPPORTED, "ac_mpe_batch: %s", g->mpe_why.c_str());
    if (mpe_lds_bytes(g->dev) > LDS_LIMIT)
        return fail(AC_ERR_UNSUPPORTED, "ac_mpe_batch: evidence and angle tables exceed LDS");
    if (B < 0) return fail(AC_ERR_INVALID_ARG, "ac_mpe_batch: B < 0");
    if (B == 0) return AC_OK;
    if (P < 1) return fail(AC_ERR_INVALID_ARG, "ac_mpe_batch: P must be >= 1 when B > 0");
    if (!param_of || !evidence || !prob_out || !mpe_out)
        return fail(AC_ERR_INVALID_ARG, "ac_mpe_batch: null param_of/evidence/prob_out/mpe_out");
    Layout L;
    make_layout(g, AC_C128, B, AC_OP_MPE, L);
    if (!ws || !fit_workspace(L, ws_bytes))
        return fail(AC_ERR_INVALID_ARG, "ac_mpe_batch: workspace of %zu bytes, need %zu (%zu for one workgroup)",
                    ws_bytes, L.total, L.tiles_off + L.per_wg_elems * L.cs);
    DeviceGuard dg(g->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *w = static_cast<uint8_t *>(ws);
    hipError_t e = launch_fixed_slots<double>(g->dev, noise, w + L.wfix_off, st);
    if (e == hipSuccess)
        e = launch_mpe(g->dev, g->mpe, L.grid, L.block, theta, param_of, P, evidence, B, w + L.wfix_off,
                       w + L.tiles_off, L.per_wg_elems, prob_out, mpe_out, st);
    if (e != hipSuccess) return fail_hip(e, "ac_mpe_batch: launch");
    return AC_OK;
}

extern "C" ac_status ac_sample(const ac_graph *g, ac_dtype dtype, const double *theta, int32_t P,
                               const double *noise, const ac_sample_cfg *cfg, uint64_t *samples,
                               uint64_t *states_out, double *cost_out, int64_t *rounds_out, void *ws,
                               size_t ws_bytes, void *stream) {
    ac_status s = check_common(g, dtype, theta, P, "ac_sample");
    if (s != AC_OK) return s;
    if (lds_bytes(g->dev) + static_cast<size_t>(g->dev.S) * (dtype == AC_C64 ? 8 : 16) >
        LDS_LIMIT)
        return fail(AC_ERR_UNSUPPORTED, "ac_sample: evidence and weight tables exceed LDS");
    if (!cfg) return fail(AC_ERR_INVALID_ARG, "ac_sample: null cfg");
    if (cfg->chains_per_param < 0 || cfg->samples_per_chain < 0 || cfg->burn_in_sweeps < 0 || cfg->thin_sweeps < 1)
        return fail(AC_ERR_INVALID_ARG, "ac_sample: bad chain schedule");
    const uint64_t sweeps = static_cast<uint64_t>(cfg->burn_in_sweeps) +
                            static_cast<uint64_t>(cfg->samples_per_chain) * static_cast<uint64_t>(cfg->thin_sweeps);
    if (static_cast<uint64_t>(cfg->first_sweep) + sweeps >= 0xFFFFFFFFull)
        return fail(AC_ERR_INVALID_ARG, "ac_sample: first_sweep + sweeps per chain must stay below 2^32 - 1");
    if (cfg->reserved != 0) return fail(AC_ERR_INVALID_ARG, "ac_sample: reserved field must be 0");
    if (cfg->chain_offset > (1ull << 62))
        return fail(AC_ERR_INVALID_ARG, "ac_sample: chain_offset above 2^62");
    if (cfg->first_var >= static_cast<uint32_t>(g->dev.n_vars))
        return fail(AC_ERR_INVALID_ARG, "ac_sample: first_var %u leaves no variable to sample", cfg->first_var);
    if (g->dev.n_qubits > 64) return fail(AC_ERR_UNSUPPORTED, "ac_sample: more than 64 output qubits");
    for (int q = 0; q < g->dev.n_qubits; ++q)
        if (g->var_offset[q] != static_cast<uint32_t>(q)) return fail(AC_ERR_UNSUPPORTED, "ac_sample: outputs must occupy bits 0..n-1");
    if (cfg->n_cost_edges < 0 || (cfg->n_cost_edges > 0 && !cfg->cost_edges))
        return fail(AC_ERR_INVALID_ARG, "ac_sample: bad cost edges");
    const int64_t total = static_cast<int64_t>(P) * cfg->chains_per_param;
    if (total == 0 || cfg->samples_per_chain == 0) return AC_OK;
    if (!samples) return fail(AC_ERR_INVALID_ARG, "ac_sample: samples is null");
    Layout L;
    make_layout(g, dtype, total, AC_OP_SAMPLE, L);
    if (!ws || !fit_workspace(L, ws_bytes))
        return fail(AC_ERR_INVALID_ARG, "ac_sample: workspace of %zu bytes, need %zu (%zu for one workgroup)",
                    ws_bytes, L.total, L.tiles_off + L.per_wg_elems * L.cs);
    DeviceGuard dg(g->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *w = static_cast<uint8_t *>(ws);
    SampleArgs a;
    a.total_chains = total;
    a.cpp = cfg->chains_per_param;
    a.spc = cfg->samples_per_chain;
    a.burn_in = cfg->burn_in_sweeps;
    a.thin = cfg->thin_sweeps;
    a.seed = cfg->seed;
    a.n_cost_edges = cfg->n_cost_edges;
    a.cost_edges = cfg->cost_edges;
    a.samples = samples;
    a.states_out = states_out;
    a.cost_out = cost_out;
    a.rounds_out = rounds_out;
    a.nwq = (g->dev.n_qubits + 63) / 64;
    a.init_states = cfg->init_states;
    a.first_sweep = cfg->first_sweep;
    a.first_var = static_cast<int32_t>(cfg->first_var);
    a.chain_offset = cfg->chain_offset;
    // QKC_SEQ_SCAN=1 decides every visit in the scan (comparisons, tests)
    const char *seq_env = std::getenv("QKC_SEQ_SCAN");
    a.seq_scan = seq_env && std::atoi(seq_env) == 1 ? 1 : 0;
    hipError_t e;
    int cpw = 0, lgrid = 0;
    const SampleKernel sk = sample_kernel(g, dtype, total);
    if (sk == SK_LDS && sample_lds_shape(g, dtype, total, cpw, lgrid)) {
        const int wpc = sample_lds_waves(g, dtype);
        e = dtype == AC_C64 ? launch_sample_lds<float>(g->dev, g->plan, cpw, wpc, lgrid, theta, noise, a, st)
                            : launch_sample_lds<double>(g->dev, g->plan, cpw, wpc, lgrid, theta, noise, a, st);
    } else if (sk == SK_STREAM) {
        if (dtype == AC_C64) {
            e = launch_fixed_slots<float>(g->dev, noise, w + L.wfix_off, st);
            if (e == hipSuccess)
                e = launch_sample_stream<float>(g->dev, g->sop, L.grid, L.block, theta, w + L.wfix_off,
                                                w + L.tiles_off,
                                                L.per_wg_elems, a, st);
        } else {
            e = launch_fixed_slots<double>(g->dev, noise, w + L.wfix_off, st);
            if (e == hipSuccess)
                e = launch_sample_stream<double>(g->dev, g->sop, L.grid, L.block, theta, w + L.wfix_off,
                                                 w + L.tiles_off,
                                                 L.per_wg_elems, a, st);
        }
    } else if (dtype == AC_C64) {
        e = launch_fixed_slots<float>(g->dev, noise, w + L.wfix_off, st);
        if (e == hipSuccess)
            e = launch_sample<float>(g->dev, L.grid, theta, w + L.wfix_off, w + L.tiles_off, L.per_wg_elems, a, st);
    } else {
        e = launch_fixed_slots<double>(g->dev, noise, w + L.wfix_off, st);
        if (e == hipSuccess)
            e = launch_sample<double>(g->dev, L.grid, theta, w + L.wfix_off, w + L.tiles_off, L.per_wg_elems, a, st);
    }
    if (e != hipSuccess) return fail_hip(e, "ac_sample: launch");
    return AC_OK;
}
