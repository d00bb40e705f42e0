// Host side of the AC evaluation library: blob parsing and validation,
// derived down-pass structures, workspace layout, argument checks and the
// extern "C" entry points declared in include/qkc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "qkc.h"
#include "qkc_internal.h"

namespace qkc {

template <typename T>
hipError_t launch_fixed_slots(const DevGraph &g, const double *noise, void *wfix, hipStream_t st);
template <typename T>
hipError_t launch_eval(const DevGraph &g, int grid, const double *theta, const int32_t *param_of,
                       const uint64_t *evidence, int64_t B, const void *wfix, void *vals, size_t per_wg_elems,
                       void *amp_out, double *prob_out, hipStream_t st);
template <typename T>
hipError_t launch_grad(const DevGraph &g, int grid, const double *theta, const int32_t *param_of,
                       const uint64_t *evidence, int64_t B, const void *wfix, void *vals, size_t per_wg_elems,
                       int mode, const void *cotangent, const double *weight, double *contrib, int P,
                       double *grad, void *amp_out, void *dfdtheta_out, void *dind_out, hipStream_t st);
template <typename T>
hipError_t launch_sample(const DevGraph &g, int grid, const double *theta, const void *wfix, void *vals,
                         size_t per_wg_elems, const SampleArgs &a, hipStream_t st);
size_t lds_bytes(const DevGraph &g, size_t csize);
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t st);

}  // namespace qkc

using namespace qkc;

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
// graph handle
// ---------------------------------------------------------------------------

struct ac_graph {
    DevGraph dev;
    void *dmem = nullptr;
    int device = 0;
    int n_cu = 0;
    ac_info_t info{};
    std::vector<uint8_t> var_dom;
    std::vector<uint32_t> var_offset;
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
    if (h[0] != 1) return fail(AC_ERR_FORMAT, "ac_load: unsupported version %u", h[0]);
    const uint32_t n_qubits = h[2], n_vars = h[3], n_words = h[4], n_angles = h[5], n_noise = h[6];
    const uint32_t n_slots = h[7], n_angle_slots = h[8], N = h[9], E = h[10], L = h[11], root = h[12];
    if (n_qubits < 1 || n_vars < n_qubits || n_vars >= (1u << 20))
        return fail(AC_ERR_FORMAT, "ac_load: bad variable counts (%u qubits, %u vars)", n_qubits, n_vars);
    if (n_words < 1 || n_words > static_cast<uint32_t>(MAX_WORDS))
        return fail(AC_ERR_FORMAT, "ac_load: n_words %u outside [1, %d]", n_words, MAX_WORDS);
    if (n_angles > static_cast<uint32_t>(MAX_ANGLES)) return fail(AC_ERR_FORMAT, "ac_load: too many angles");
    if (n_angle_slots > n_slots || n_angle_slots > static_cast<uint32_t>(MAX_ANGLE_SLOTS))
        return fail(AC_ERR_FORMAT, "ac_load: bad angle-slot count %u", n_angle_slots);
    if (N < 1 || L < 1 || L > N || E < N || root >= N)
        return fail(AC_ERR_FORMAT, "ac_load: bad DAG sizes (N=%u E=%u L=%u root=%u)", N, E, L, root);

    const uint8_t *var_dom = rd.take<uint8_t>(n_vars);
    const uint8_t *var_kind = rd.take_packed<uint8_t>(n_vars);
    const uint32_t *var_off = rd.take<uint32_t>(n_vars);
    const double *noise_def = rd.take<double>(n_noise);
    const SlotDesc *slots = rd.take_packed<SlotDesc>(n_slots);
    const uint8_t *op = rd.take_packed<uint8_t>(N);
    const uint32_t *row_ptr = rd.take<uint32_t>(N + 1);
    const uint32_t *col = rd.take<uint32_t>(E);
    const uint32_t *level_ptr = rd.take<uint32_t>(L + 1);
    if (!rd.ok) return fail(AC_ERR_FORMAT, "ac_load: blob truncated");

    // ---- evidence variables
    std::vector<uint32_t> ind_base(n_vars + 1, 0), var_field(n_vars);
    for (uint32_t v = 0; v < n_vars; ++v) {
        const uint32_t d = var_dom[v];
        if (d < 2 || d > static_cast<uint32_t>(MAX_DOM)) return fail(AC_ERR_FORMAT, "ac_load: variable %u domain %u", v, d);
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
    for (uint32_t m = 0; m < n_noise; ++m)
        if (!(noise_def[m] >= 0.0 && noise_def[m] <= 1.0)) return fail(AC_ERR_FORMAT, "ac_load: noise %u outside [0,1]", m);

    // ---- DAG
    if (row_ptr[0] != 0 || row_ptr[N] != E) return fail(AC_ERR_FORMAT, "ac_load: row_ptr ends");
    if (level_ptr[0] != 0 || level_ptr[L] != N) return fail(AC_ERR_FORMAT, "ac_load: level_ptr ends");
    std::vector<uint32_t> level(N);
    uint32_t max_width = 0;
    for (uint32_t l = 0; l < L; ++l) {
        if (level_ptr[l + 1] <= level_ptr[l]) return fail(AC_ERR_FORMAT, "ac_load: empty level %u", l);
        max_width = std::max(max_width, level_ptr[l + 1] - level_ptr[l]);
        for (uint32_t i = level_ptr[l]; i < level_ptr[l + 1]; ++i) level[i] = l;
    }
    if (level[root] != L - 1 || level_ptr[L - 1] != N - 1)
        return fail(AC_ERR_FORMAT, "ac_load: the root must be the only node of the top level");
    std::vector<uint32_t> dcol(E), edge_parent(E);
    std::vector<uint32_t> n_par(N, 0), n_leafpar(n_ind + n_slots, 0);
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
                return fail(AC_ERR_FORMAT, "ac_load: edge %u bad tag", e);
            }
        }
    }
    // parent CSR of internal nodes and of leaves (edges in increasing order)
    std::vector<uint32_t> par_ptr(N + 1, 0), leaf_ptr(n_ind + n_slots + 1, 0);
    for (uint32_t i = 0; i < N; ++i) par_ptr[i + 1] = par_ptr[i] + n_par[i];
    for (uint32_t i = 0; i < n_ind + n_slots; ++i) leaf_ptr[i + 1] = leaf_ptr[i] + n_leafpar[i];
    std::vector<uint32_t> par_edge(par_ptr[N]), leaf_edge(leaf_ptr[n_ind + n_slots]);
    {
        std::vector<uint32_t> fp(par_ptr.begin(), par_ptr.end() - 1), fl(leaf_ptr.begin(), leaf_ptr.end() - 1);
        for (uint32_t e = 0; e < E; ++e) {
            const uint32_t r = col[e], tag = r >> 30, x = r & REF_MASK;
            if (tag == TAG_NODE) par_edge[fp[x]++] = e;
            else if (tag == TAG_IND) leaf_edge[fl[ind_base[x & 0xffffffu] + (x >> 24)]++] = e;
            else leaf_edge[fl[n_ind + x]++] = e;
        }
    }

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
    inf.root = d.root;
    inf.device = device;
    inf.n_prod_flops = flops;
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

constexpr size_t WS_CAP = static_cast<size_t>(48) << 30;   // cap on per-call tile buffers
constexpr size_t LDS_LIMIT = 64 * 1024;                     // dynamic LDS per workgroup
constexpr int WG_PER_CU = 4;

struct Layout {
    size_t wfix_off = 0, contrib_off = 0, tiles_off = 0, total = 0;
    size_t per_wg_elems = 0;   // complex elements per workgroup buffer
    int grid = 0;
};

bool make_layout(const ac_graph *g, ac_dtype dt, int64_t batch, int op, Layout &out) {
    if (!g || batch < 0 || (dt != AC_C64 && dt != AC_C128) || op < 0 || op > 2) return false;
    const DevGraph &d = g->dev;
    const size_t cs = dt == AC_C64 ? 8 : 16;
    size_t rows = 0;
    if (op == AC_OP_EVAL) rows = d.N;
    else if (op == AC_OP_GRAD) rows = 2 * static_cast<size_t>(d.N) + d.S_ang;
    else rows = 2 * static_cast<size_t>(d.N) + d.n_ind;
    const size_t per_wg = rows * WAVE;
    int64_t tiles = (batch + WAVE - 1) / WAVE;
    int64_t grid = std::min<int64_t>(tiles, static_cast<int64_t>(g->n_cu) * WG_PER_CU);
    const int64_t cap = std::max<int64_t>(1, static_cast<int64_t>(WS_CAP / (per_wg * cs)));
    grid = std::min(grid, cap);
    if (batch > 0 && grid < 1) grid = 1;
    Layout L;
    size_t off = 0;
    L.wfix_off = off;
    off += align256(static_cast<size_t>(std::max(d.S, 1)) * cs);
    L.contrib_off = off;
    if (op == AC_OP_GRAD) off += align256(static_cast<size_t>(std::max<int64_t>(batch, 1)) * std::max(d.K, 1) * 8);
    L.tiles_off = off;
    off += align256(static_cast<size_t>(grid) * per_wg * cs);
    L.total = off;
    L.per_wg_elems = per_wg;
    L.grid = static_cast<int>(grid);
    out = L;
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

extern "C" ac_status ac_eval_batch(const ac_graph *g, ac_dtype dtype, const double *theta, int32_t P,
                                   const double *noise, const int32_t *param_of, const uint64_t *evidence,
                                   int64_t B, void *amp_out, double *prob_out, void *ws, size_t ws_bytes,
                                   void *stream) {
    ac_status s = check_common(g, dtype, theta, P, "ac_eval_batch");
    if (s != AC_OK) return s;
    if (lds_bytes(g->dev, dtype == AC_C64 ? 8 : 16) > LDS_LIMIT)
        return fail(AC_ERR_UNSUPPORTED, "ac_eval_batch: evidence and angle tables exceed LDS");
    if (B < 0) return fail(AC_ERR_INVALID_ARG, "ac_eval_batch: B < 0");
    if (B == 0) return AC_OK;
    if (P < 1) return fail(AC_ERR_INVALID_ARG, "ac_eval_batch: P must be >= 1 when B > 0");
    if (!param_of || !evidence || !amp_out) return fail(AC_ERR_INVALID_ARG, "ac_eval_batch: null param_of/evidence/amp_out");
    Layout L;
    make_layout(g, dtype, B, AC_OP_EVAL, L);
    if (!ws || ws_bytes < L.total)
        return fail(AC_ERR_INVALID_ARG, "ac_eval_batch: workspace of %zu bytes, need %zu", ws_bytes, L.total);
    DeviceGuard dg(g->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *w = static_cast<uint8_t *>(ws);
    hipError_t e;
    if (dtype == AC_C64) {
        e = launch_fixed_slots<float>(g->dev, noise, w + L.wfix_off, st);
        if (e == hipSuccess)
            e = launch_eval<float>(g->dev, L.grid, theta, param_of, evidence, B, w + L.wfix_off, w + L.tiles_off,
                                   L.per_wg_elems, amp_out, prob_out, st);
    } else {
        e = launch_fixed_slots<double>(g->dev, noise, w + L.wfix_off, st);
        if (e == hipSuccess)
            e = launch_eval<double>(g->dev, L.grid, theta, param_of, evidence, B, w + L.wfix_off, w + L.tiles_off,
                                    L.per_wg_elems, amp_out, prob_out, st);
    }
    if (e != hipSuccess) return fail_hip(e, "ac_eval_batch: launch");
    return AC_OK;
}

extern "C" ac_status ac_grad_batch(const ac_graph *g, ac_dtype dtype, const double *theta, int32_t P,
                                   const double *noise, const int32_t *param_of, const uint64_t *evidence,
                                   int64_t B, int mode, const void *cotangent, const double *weight,
                                   double *grad_theta, void *amp_out, void *dfdtheta_out, void *dind_out,
                                   void *ws, size_t ws_bytes, void *stream) {
    ac_status s = check_common(g, dtype, theta, P, "ac_grad_batch");
    if (s != AC_OK) return s;
    if (lds_bytes(g->dev, dtype == AC_C64 ? 8 : 16) > LDS_LIMIT)
        return fail(AC_ERR_UNSUPPORTED, "ac_grad_batch: evidence and angle tables exceed LDS");
    if (B < 0) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: B < 0");
    if (mode < 0 || mode > 2) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: bad mode %d", mode);
    if (mode == AC_GRAD_COTANGENT && B > 0 && !cotangent) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: cotangent is null");
    if (mode != AC_GRAD_COTANGENT && B > 0 && !weight) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: weight is null");
    if (g->dev.K > 0 && P > 0 && !grad_theta) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: grad_theta is null");
    if (B > 0 && (!param_of || !evidence)) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: null param_of/evidence");
    if (B > 0 && P < 1) return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: P must be >= 1 when B > 0");
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
    if (!ws || ws_bytes < L.total)
        return fail(AC_ERR_INVALID_ARG, "ac_grad_batch: workspace of %zu bytes, need %zu", ws_bytes, L.total);
    uint8_t *w = static_cast<uint8_t *>(ws);
    double *contrib = reinterpret_cast<double *>(w + L.contrib_off);
    hipError_t e;
    if (dtype == AC_C64) {
        e = launch_fixed_slots<float>(g->dev, noise, w + L.wfix_off, st);
        if (e == hipSuccess)
            e = launch_grad<float>(g->dev, L.grid, theta, param_of, evidence, B, w + L.wfix_off, w + L.tiles_off,
                                   L.per_wg_elems, mode, cotangent, weight, contrib, P, grad_theta, amp_out,
                                   dfdtheta_out, dind_out, st);
    } else {
        e = launch_fixed_slots<double>(g->dev, noise, w + L.wfix_off, st);
        if (e == hipSuccess)
            e = launch_grad<double>(g->dev, L.grid, theta, param_of, evidence, B, w + L.wfix_off, w + L.tiles_off,
                                    L.per_wg_elems, mode, cotangent, weight, contrib, P, grad_theta, amp_out,
                                    dfdtheta_out, dind_out, st);
    }
    if (e != hipSuccess) return fail_hip(e, "ac_grad_batch: launch");
    return AC_OK;
}

extern "C" ac_status ac_sample(const ac_graph *g, ac_dtype dtype, const double *theta, int32_t P,
                               const double *noise, const ac_sample_cfg *cfg, uint64_t *samples,
                               uint64_t *states_out, double *cost_out, int64_t *rounds_out, void *ws,
                               size_t ws_bytes, void *stream) {
    ac_status s = check_common(g, dtype, theta, P, "ac_sample");
    if (s != AC_OK) return s;
    if (lds_bytes(g->dev, dtype == AC_C64 ? 8 : 16) > LDS_LIMIT)
        return fail(AC_ERR_UNSUPPORTED, "ac_sample: evidence and angle tables exceed LDS");
    if (!cfg) return fail(AC_ERR_INVALID_ARG, "ac_sample: null cfg");
    if (cfg->chains_per_param < 0 || cfg->samples_per_chain < 0 || cfg->burn_in_sweeps < 0 || cfg->thin_sweeps < 1)
        return fail(AC_ERR_INVALID_ARG, "ac_sample: bad chain schedule");
    const uint64_t sweeps = static_cast<uint64_t>(cfg->burn_in_sweeps) +
                            static_cast<uint64_t>(cfg->samples_per_chain) * static_cast<uint64_t>(cfg->thin_sweeps);
    if (sweeps >= 0xFFFFFFFFull) return fail(AC_ERR_INVALID_ARG, "ac_sample: too many sweeps per chain");
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
    if (!ws || ws_bytes < L.total)
        return fail(AC_ERR_INVALID_ARG, "ac_sample: workspace of %zu bytes, need %zu", ws_bytes, L.total);
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
    hipError_t e;
    if (dtype == AC_C64) {
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
