// Plain CPU evaluator of the compiled arithmetic circuits (include/qkc_cpu.h):
// complex128, node by node in the blob's level order, OpenMP over batch
// elements and chains.  A baseline for the GPU library, with its own blob
// reader, weights, passes and sampler.
#include "qkc_cpu.h"

#include <omp.h>

#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace {

using cd = std::complex<double>;

thread_local std::string last_error;

int fail(const char *fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    last_error = buf;
    return 1;
}

// blob reference tags (bits 31..30) and the slot kinds of the blob format
enum : uint32_t { R_NODE = 0, R_IND = 1, R_SLOT = 2, R_SEL = 3 };
constexpr uint32_t IDX = 0x3fffffffu;
constexpr uint32_t NONE = 0xffffffffu;

struct SlotRec {
    uint8_t base, coef;
    int32_t index;
    double scale, re, im;
};

struct Var {
    uint32_t word, shift, mask, dom;
};

}  // namespace

struct qkc_cpu {
    uint32_t n_qubits = 0, n_vars = 0, n_words = 0, n_angles = 0, n_noise = 0, n_slots = 0, n_sel = 0;
    uint32_t N = 0, E = 0, root = 0;
    std::vector<Var> vars;
    std::vector<uint32_t> ind_base;        // first indicator index of each variable
    std::vector<double> noise_default;
    std::vector<SlotRec> slots;
    std::vector<uint32_t> sel_var, sel_slot;   // selector q: variable, slot per value (4)
    std::vector<uint8_t> op;
    std::vector<uint32_t> row_ptr, col;
};

namespace {

struct Reader {
    const uint8_t *p;
    size_t n, pos = 0;
    bool ok = true;
    const uint8_t *take(size_t bytes, bool align) {
        if (align) pos = (pos + 7) & ~size_t{7};
        if (pos > n || bytes > n - pos) {
            ok = false;
            return nullptr;
        }
        const uint8_t *r = p + pos;
        pos += bytes;
        return r;
    }
};

template <typename T>
T rd(const uint8_t *p) {
    T v;
    std::memcpy(&v, p, sizeof(T));
    return v;
}

// value of a weight slot for one row of angles and the noise strengths
cd slot_value(const SlotRec &s, const double *th, const double *nz) {
    double re = 0.0, im = 0.0;
    const double a = th && s.base >= 1 && s.base <= 4 ? 0.5 * s.scale * th[s.index] : 0.0;
    switch (s.base) {
        case 0: re = s.re; im = s.im; break;
        case 1: re = std::cos(a); break;
        case 2: re = std::sin(a); break;
        case 3: re = std::cos(a); im = -std::sin(a); break;
        case 4: re = std::cos(a); im = std::sin(a); break;
        case 5: re = std::sqrt(1.0 - nz[s.index]); break;
        case 6: re = std::sqrt(nz[s.index] / 3.0); break;
        case 7: re = std::sqrt(nz[s.index]); break;
        default: break;
    }
    const cd v(re, im);
    switch (s.coef) {
        case 1: return -v;
        case 2: return cd(0.0, 1.0) * v;
        case 3: return cd(0.0, -1.0) * v;
        default: return v;
    }
}

inline uint32_t field(const qkc_cpu &ac, const uint64_t *ev, uint32_t v) {
    const Var &x = ac.vars[v];
    return static_cast<uint32_t>((ev[x.word] >> x.shift) & x.mask);
}

// per-thread scratch of one evaluation
struct Work {
    std::vector<cd> w, val, adj, D, pre;
    void size(const qkc_cpu &ac) {
        w.assign(ac.n_slots, cd());
        val.assign(ac.N, cd());
        adj.assign(ac.N, cd());
        D.assign(ac.ind_base[ac.n_vars], cd());
    }
};

void weights(const qkc_cpu &ac, const double *th, const double *nz, Work &k) {
    for (uint32_t s = 0; s < ac.n_slots; ++s) k.w[s] = slot_value(ac.slots[s], th, nz);
}

inline cd leaf(const qkc_cpu &ac, const uint64_t *ev, const Work &k, uint32_t r) {
    const uint32_t t = r >> 30, x = r & IDX;
    if (t == R_NODE) return k.val[x];
    if (t == R_IND) return field(ac, ev, x & 0xffffffu) == (x >> 24) ? cd(1.0, 0.0) : cd();
    if (t == R_SLOT) return k.w[x];
    const uint32_t u = field(ac, ev, ac.sel_var[x]);
    const uint32_t sl = u < 4 ? ac.sel_slot[4 * x + u] : NONE;
    return sl == NONE ? cd() : k.w[sl];
}

// upward pass: every node value, in level order
void upward(const qkc_cpu &ac, const uint64_t *ev, Work &k) {
    for (uint32_t i = 0; i < ac.N; ++i) {
        const bool prod = ac.op[i] != 0;
        cd acc = prod ? cd(1.0, 0.0) : cd();
        for (uint32_t e = ac.row_ptr[i]; e < ac.row_ptr[i + 1]; ++e) {
            const cd v = leaf(ac, ev, k, ac.col[e]);
            acc = prod ? acc * v : acc + v;
        }
        k.val[i] = acc;
    }
}

// downward pass: adj[i] = d root / d node i, and D[ind_base[v] + u] =
// d root / d lambda_{v=u}; a product passes adj times the product of its
// other children (prefix and suffix products, no division)
void downward(const qkc_cpu &ac, const uint64_t *ev, Work &k) {
    std::fill(k.adj.begin(), k.adj.end(), cd());
    std::fill(k.D.begin(), k.D.end(), cd());
    k.adj[ac.root] = cd(1.0, 0.0);
    for (uint32_t i = ac.N; i-- > 0;) {
        const cd a = k.adj[i];
        const uint32_t e0 = ac.row_ptr[i], e1 = ac.row_ptr[i + 1], n = e1 - e0;
        if (ac.op[i] != 0) {
            k.pre.resize(n + 1);
            k.pre[0] = cd(1.0, 0.0);
            for (uint32_t j = 0; j < n; ++j) k.pre[j + 1] = k.pre[j] * leaf(ac, ev, k, ac.col[e0 + j]);
        }
        cd suf(1.0, 0.0);
        for (uint32_t j = n; j-- > 0;) {
            const uint32_t r = ac.col[e0 + j], t = r >> 30, x = r & IDX;
            const cd term = ac.op[i] != 0 ? a * k.pre[j] * suf : a;
            if (ac.op[i] != 0) suf *= leaf(ac, ev, k, r);
            if (t == R_NODE) {
                k.adj[x] += term;
            } else if (t == R_IND) {
                k.D[ac.ind_base[x & 0xffffffu] + (x >> 24)] += term;
            } else if (t == R_SEL) {
                const uint32_t v = ac.sel_var[x];
                for (uint32_t u = 0; u < 4 && u < ac.vars[v].dom; ++u) {
                    const uint32_t sl = ac.sel_slot[4 * x + u];
                    if (sl != NONE) k.D[ac.ind_base[v] + u] += term * k.w[sl];
                }
            }
        }
    }
}

// SplitMix64 finaliser of z + golden gamma (Steele, Lea and Flood, OOPSLA 2014)
inline uint64_t mix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

inline double uniform(uint64_t seed, uint64_t chain, uint64_t sweep, uint64_t var) {
    const uint64_t top = mix(seed ^ mix(chain ^ mix((sweep << 20) ^ var)));
    return static_cast<double>(top >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace

extern "C" const char *qkc_cpu_last_error(void) { return last_error.c_str(); }

extern "C" int qkc_cpu_load(const void *blob, size_t nbytes, qkc_cpu **out) {
    if (!blob || !out) return fail("qkc_cpu_load: null argument");
    *out = nullptr;
    Reader r{static_cast<const uint8_t *>(blob), nbytes};
    const uint8_t *hdr = r.take(8 + 14 * 4, false);
    if (!r.ok) return fail("qkc_cpu_load: short blob");
    static const uint8_t magic[8] = {'Q', 'K', 'C', 'A', 'C', 0, 0, 1};
    if (std::memcmp(hdr, magic, 8) != 0) return fail("qkc_cpu_load: bad magic");
    uint32_t h[14];
    for (int i = 0; i < 14; ++i) h[i] = rd<uint32_t>(hdr + 8 + 4 * i);
    if (h[0] != 2) return fail("qkc_cpu_load: version %u", h[0]);
    auto *ac = new qkc_cpu();
    auto bad = [&](const char *what) {
        delete ac;
        return fail("qkc_cpu_load: %s", what);
    };
    ac->n_qubits = h[2];
    ac->n_vars = h[3];
    ac->n_words = h[4];
    ac->n_angles = h[5];
    ac->n_noise = h[6];
    ac->n_slots = h[7];
    ac->N = h[9];
    ac->E = h[10];
    const uint32_t L = h[11];
    ac->root = h[12];
    ac->n_sel = h[13];
    if (ac->n_vars < ac->n_qubits || ac->n_vars >= (1u << 24) || ac->n_words < 1 || ac->N < 1 || ac->root >= ac->N ||
        ac->E < ac->N || L < 1)
        return bad("sizes");
    const uint8_t *dom = r.take(ac->n_vars, true);
    r.take(ac->n_vars, false);                       // variable kinds (not needed here)
    const uint8_t *off = r.take(4ull * ac->n_vars, true);
    const uint8_t *nz = r.take(8ull * ac->n_noise, true);
    const uint8_t *sl = r.take(32ull * ac->n_slots, false);
    const uint8_t *se = r.take(20ull * ac->n_sel, false);
    const uint8_t *op = r.take(ac->N, false);
    const uint8_t *rp = r.take(4ull * (ac->N + 1), true);
    const uint8_t *cl = r.take(4ull * ac->E, true);
    if (!r.ok) return bad("truncated");
    ac->ind_base.assign(ac->n_vars + 1, 0);
    for (uint32_t v = 0; v < ac->n_vars; ++v) {
        const uint32_t d = dom[v], o = rd<uint32_t>(off + 4 * v);
        uint32_t width = 0;
        while ((1u << width) < d) ++width;
        if (d < 2 || width > 4 || o / 64 >= ac->n_words || o % 64 + width > 64) return bad("variable field");
        ac->vars.push_back({o / 64, o % 64, (1u << width) - 1u, d});
        ac->ind_base[v + 1] = ac->ind_base[v] + d;
    }
    for (uint32_t m = 0; m < ac->n_noise; ++m) ac->noise_default.push_back(rd<double>(nz + 8 * m));
    for (uint32_t s = 0; s < ac->n_slots; ++s) {
        const uint8_t *q = sl + 32 * s;
        SlotRec x{q[0], q[1], rd<int32_t>(q + 4), rd<double>(q + 8), rd<double>(q + 16), rd<double>(q + 24)};
        if (x.base > 7 || x.coef > 3) return bad("slot kind");
        if (x.base >= 1 && x.base <= 4 && (x.index < 0 || static_cast<uint32_t>(x.index) >= ac->n_angles))
            return bad("slot angle");
        if (x.base >= 5 && (x.index < 0 || static_cast<uint32_t>(x.index) >= ac->n_noise)) return bad("slot noise");
        ac->slots.push_back(x);
    }
    for (uint32_t q = 0; q < ac->n_sel; ++q) {
        const uint32_t v = rd<uint32_t>(se + 20 * q);
        if (v >= ac->n_vars) return bad("selector variable");
        ac->sel_var.push_back(v);
        for (int u = 0; u < 4; ++u) {
            const uint32_t s = rd<uint32_t>(se + 20 * q + 4 + 4 * u);
            if (s != NONE && s >= ac->n_slots) return bad("selector slot");
            ac->sel_slot.push_back(s);
        }
    }
    ac->op.assign(op, op + ac->N);
    for (uint32_t i = 0; i <= ac->N; ++i) ac->row_ptr.push_back(rd<uint32_t>(rp + 4 * i));
    if (ac->row_ptr[0] != 0 || ac->row_ptr[ac->N] != ac->E) return bad("row_ptr");
    for (uint32_t i = 0; i < ac->N; ++i)
        if (ac->row_ptr[i + 1] < ac->row_ptr[i]) return bad("row_ptr order");
    for (uint32_t e = 0; e < ac->E; ++e) ac->col.push_back(rd<uint32_t>(cl + 4 * e));
    for (uint32_t i = 0; i < ac->N; ++i)
        for (uint32_t e = ac->row_ptr[i]; e < ac->row_ptr[i + 1]; ++e) {
            const uint32_t c = ac->col[e], t = c >> 30, x = c & IDX;
            const bool ok = t == R_NODE   ? x < i
                            : t == R_IND  ? (x & 0xffffffu) < ac->n_vars && (x >> 24) < ac->vars[x & 0xffffffu].dom
                            : t == R_SLOT ? x < ac->n_slots
                                          : x < ac->n_sel;
            if (!ok) return bad("child reference");
        }
    *out = ac;
    return 0;
}

extern "C" void qkc_cpu_free(qkc_cpu *ac) { delete ac; }

extern "C" int qkc_cpu_info(const qkc_cpu *ac, int32_t *n_internal, int64_t *n_edges, int32_t *n_vars,
                            int32_t *n_words, int32_t *n_angles, int32_t *n_qubits) {
    if (!ac) return fail("qkc_cpu_info: null handle");
    if (n_internal) *n_internal = static_cast<int32_t>(ac->N);
    if (n_edges) *n_edges = ac->E;
    if (n_vars) *n_vars = static_cast<int32_t>(ac->n_vars);
    if (n_words) *n_words = static_cast<int32_t>(ac->n_words);
    if (n_angles) *n_angles = static_cast<int32_t>(ac->n_angles);
    if (n_qubits) *n_qubits = static_cast<int32_t>(ac->n_qubits);
    return 0;
}

extern "C" int qkc_cpu_eval(const qkc_cpu *ac, const double *theta, int32_t P, const double *noise,
                            const int32_t *param_of, const uint64_t *evidence, int64_t B, double *amp_out,
                            int threads) {
    if (!ac || B < 0 || (B > 0 && (!param_of || !evidence || !amp_out || P < 1)) ||
        (ac->n_angles > 0 && P > 0 && !theta))
        return fail("qkc_cpu_eval: invalid arguments");
    const double *nz = noise ? noise : ac->noise_default.data();
    int err = 0;
#pragma omp parallel num_threads(threads > 0 ? threads : omp_get_max_threads())
    {
        Work k;
        k.size(*ac);
        int32_t have = -1;
#pragma omp for schedule(static)
        for (int64_t b = 0; b < B; ++b) {
            const int32_t p = param_of[b];
            if (p < 0 || p >= P) {
#pragma omp atomic write
                err = 1;
                amp_out[2 * b] = amp_out[2 * b + 1] = NAN;
                continue;
            }
            if (p != have) {
                weights(*ac, theta + static_cast<int64_t>(p) * ac->n_angles, nz, k);
                have = p;
            }
            upward(*ac, evidence + b * ac->n_words, k);
            amp_out[2 * b] = k.val[ac->root].real();
            amp_out[2 * b + 1] = k.val[ac->root].imag();
        }
    }
    return err ? fail("qkc_cpu_eval: param_of entries outside [0, P)") : 0;
}

extern "C" int qkc_cpu_sample(const qkc_cpu *ac, const double *theta, int32_t P, const double *noise,
                              int32_t chains_per_param, int32_t samples_per_chain, int32_t burn_in, int32_t thin,
                              uint64_t seed, uint64_t *samples_out, uint64_t *states_out, int64_t *rounds_out,
                              int threads) {
    if (!ac || P < 0 || chains_per_param < 0 || samples_per_chain < 0 || burn_in < 0 || thin < 1 ||
        ac->n_qubits > 64 || (ac->n_angles > 0 && P > 0 && !theta) || !samples_out)
        return fail("qkc_cpu_sample: invalid arguments");
    for (uint32_t q = 0; q < ac->n_qubits; ++q)
        if (ac->vars[q].word != 0 || ac->vars[q].shift != q) return fail("qkc_cpu_sample: outputs must be bits 0..n-1");
    const double *nz = noise ? noise : ac->noise_default.data();
    const int64_t total = static_cast<int64_t>(P) * chains_per_param;
    const int64_t S = static_cast<int64_t>(chains_per_param) * samples_per_chain;
    const uint32_t sweeps = static_cast<uint32_t>(burn_in) + static_cast<uint32_t>(samples_per_chain) * thin;
    const uint64_t xmask = ac->n_qubits >= 64 ? ~0ull : ((1ull << ac->n_qubits) - 1ull);
    const uint32_t V = ac->n_vars;
#pragma omp parallel num_threads(threads > 0 ? threads : omp_get_max_threads())
    {
        Work k;
        k.size(*ac);
        std::vector<uint64_t> ev(ac->n_words);
        int32_t have = -1;
#pragma omp for schedule(dynamic, 16)
        for (int64_t ch = 0; ch < total; ++ch) {
            const int32_t p = static_cast<int32_t>(ch / chains_per_param);
            const int64_t c = ch % chains_per_param;
            if (p != have) {
                weights(*ac, theta + static_cast<int64_t>(p) * ac->n_angles, nz, k);
                have = p;
            }
            std::fill(ev.begin(), ev.end(), 0ull);
            for (uint32_t q = 0; q < ac->n_qubits; ++q)
                if (uniform(seed, static_cast<uint64_t>(ch), 0xFFFFFFFFull, q) < 0.5) ev[0] |= 1ull << q;
            uint32_t pos = 0, sweep = 0;
            int64_t emitted = 0, rounds = 0;
            while (sweep < sweeps) {
                upward(*ac, ev.data(), k);
                downward(*ac, ev.data(), k);
                ++rounds;
                for (;;) {                              // visits until the first change
                    const uint32_t v = pos;
                    const uint32_t base = ac->ind_base[v], dom = ac->vars[v].dom;
                    const uint32_t cur = field(*ac, ev.data(), v);
                    double tot = 0.0;
                    for (uint32_t u = 0; u < dom; ++u) tot += std::norm(k.D[base + u]);
                    uint32_t pick = cur;
                    if (tot > 0.0) {
                        const double target = uniform(seed, static_cast<uint64_t>(ch), sweep, v) * tot;
                        double acc = 0.0;
                        int last = -1, chosen = -1;
                        for (uint32_t u = 0; u < dom; ++u) {
                            const double w = std::norm(k.D[base + u]);
                            acc += w;
                            if (w > 0.0) last = static_cast<int>(u);
                            if (target < acc) {
                                chosen = static_cast<int>(u);
                                break;
                            }
                        }
                        if (chosen < 0) chosen = last;
                        if (chosen >= 0) pick = static_cast<uint32_t>(chosen);
                    }
                    const bool changed = pick != cur;
                    if (changed) {
                        const Var &x = ac->vars[v];
                        ev[x.word] = (ev[x.word] & ~(static_cast<uint64_t>(x.mask) << x.shift)) |
                                     (static_cast<uint64_t>(pick) << x.shift);
                    }
                    if (++pos == V) {
                        pos = 0;
                        ++sweep;
                        if (sweep > static_cast<uint32_t>(burn_in) &&
                            (sweep - static_cast<uint32_t>(burn_in)) % static_cast<uint32_t>(thin) == 0u) {
                            const int64_t idx = static_cast<int64_t>(p) * S + c * samples_per_chain + emitted;
                            samples_out[idx] = ev[0] & xmask;
                            if (states_out)
                                for (uint32_t w = 0; w < ac->n_words; ++w) states_out[idx * ac->n_words + w] = ev[w];
                            ++emitted;
                        }
                        if (sweep >= sweeps) break;
                    }
                    if (changed) break;
                }
            }
            if (rounds_out) rounds_out[ch] = rounds;
        }
    }
    return 0;
}
