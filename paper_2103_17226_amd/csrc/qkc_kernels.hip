// HIP kernels of the batched arithmetic-circuit evaluator (gfx950).
//
// Execution model: one workgroup of 4 wavefronts owns a tile of 64 batch
// elements; lane = batch element, so every node's value for the tile is one
// coalesced 512-byte (complex64) or 1 KiB (complex128) row.  The four waves
// split each DAG level's nodes and meet at a barrier between levels (the DAG
// is level-ordered on the host).  Node descriptors and child references are
// wave-uniform and come in through scalar loads; indicator leaves are decoded
// from the tile's evidence words in LDS, angle-dependent weights are computed
// per lane in FP64 and staged in LDS, and the remaining weights are computed
// once per call and read through scalar loads.  Grids are persistent: a
// workgroup walks tiles (or Gibbs chains) until the batch is done.
#include <hip/hip_runtime.h>

#include "qkc_internal.h"

namespace qkc {

template <typename T>
struct cplx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
    return {a.re + b.re, a.im + b.im};
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}

// ---------------------------------------------------------------------------
// weights (FP64, then rounded to the pass dtype)
// ---------------------------------------------------------------------------

__device__ inline void apply_coef(uint8_t coef, double &re, double &im) {
    double r = re, i = im;
    switch (coef) {
        case 1: re = -r; im = -i; break;
        case 2: re = -i; im = r; break;     // i * (r + i i)
        case 3: re = i; im = -r; break;     // -i * (r + i i)
        default: break;
    }
}

__device__ inline void slot_value(const SlotDesc &s, const double *theta_row, const double *noise,
                                  double &re, double &im) {
    re = 0.0;
    im = 0.0;
    switch (s.base) {
        case B_CONST: re = s.re; im = s.im; break;
        case B_COS: re = cos(0.5 * s.scale * theta_row[s.index]); break;
        case B_SIN: re = sin(0.5 * s.scale * theta_row[s.index]); break;
        case B_EXPM: {
            double a = 0.5 * s.scale * theta_row[s.index];
            re = cos(a); im = -sin(a);
        } break;
        case B_EXPP: {
            double a = 0.5 * s.scale * theta_row[s.index];
            re = cos(a); im = sin(a);
        } break;
        case B_SQRT_1MP: re = sqrt(1.0 - noise[s.index]); break;
        case B_SQRT_P3: re = sqrt(noise[s.index] / 3.0); break;
        case B_SQRT_P: re = sqrt(noise[s.index]); break;
        default: break;
    }
    apply_coef(s.coef, re, im);
}

// d(slot value)/d theta[s.index] for an angle slot.
__device__ inline void slot_dvalue(const SlotDesc &s, const double *theta_row, double &re,
                                   double &im) {
    double h = 0.5 * s.scale;
    double a = h * theta_row[s.index];
    re = 0.0;
    im = 0.0;
    switch (s.base) {
        case B_COS: re = -h * sin(a); break;
        case B_SIN: re = h * cos(a); break;
        case B_EXPM: re = -h * sin(a); im = -h * cos(a); break;   // -i h e^{-ia}
        case B_EXPP: re = -h * sin(a); im = h * cos(a); break;    // +i h e^{+ia}
        default: break;
    }
    apply_coef(s.coef, re, im);
}

// One thread per slot: weights that do not depend on theta.
template <typename T>
__global__ void k_fixed_slots(DevGraph g, const double *noise, cplx<T> *wfix) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.S) return;
    const double *nz = noise ? noise : g.noise_default;
    double re = 0.0, im = 0.0;
    if (s >= g.S_ang) slot_value(g.slots[s], nullptr, nz, re, im);
    wfix[s] = {static_cast<T>(re), static_cast<T>(im)};
}

// ---------------------------------------------------------------------------
// tile context
// ---------------------------------------------------------------------------

template <typename T>
struct Tile {
    DevGraph g;
    cplx<T> *val;            // [N][64] node values of this tile (global)
    const uint64_t *ev;      // [W][64] evidence words (LDS)
    const cplx<T> *ang;      // [S_ang][64] angle weights (LDS)
    const cplx<T> *wfix;     // [S] fixed weights (global, uniform reads)
    int lane;

    __device__ __forceinline__ bool ind_hit(uint32_t r) const {
        uint32_t u = (r >> 26) & 15u;
        uint32_t width = ((r >> 24) & 3u) + 1u;
        uint32_t word = (r >> 6) & 0x3ffffu;
        uint32_t shift = r & 63u;
        uint64_t x = (ev[word * WAVE + lane] >> shift) & ((1ull << width) - 1ull);
        return x == static_cast<uint64_t>(u);
    }

    __device__ __forceinline__ cplx<T> slot(uint32_t s) const {
        if (s < static_cast<uint32_t>(g.S_ang)) return ang[s * WAVE + lane];
        return wfix[s];
    }

    // value of a child reference (leaves computed on the fly)
    __device__ __forceinline__ cplx<T> child(uint32_t r) const {
        uint32_t tag = r >> 30;
        if (tag == TAG_NODE) return val[(r & REF_MASK) * WAVE + lane];
        if (tag == TAG_IND) return {ind_hit(r) ? T(1) : T(0), T(0)};
        return slot(r & REF_MASK);
    }

    // Sum nodes accumulate in FP64 (for the complex64 path too: wide sums
    // would otherwise lose ~k * 2^-24 relative accuracy); products run in T.
    __device__ __forceinline__ cplx<T> eval_node(uint32_t i) const {
        const uint32_t e0 = g.row_ptr[i], e1 = g.row_ptr[i + 1];
        if (g.op[i] == 0) {
            double sr = 0.0, si = 0.0;
            for (uint32_t e = e0; e < e1; ++e) {
                const uint32_t r = g.col[e];
                const uint32_t tag = r >> 30;
                if (tag == TAG_IND) {
                    sr += ind_hit(r) ? 1.0 : 0.0;
                    continue;
                }
                const cplx<T> v = (tag == TAG_NODE) ? val[(r & REF_MASK) * WAVE + lane] : slot(r & REF_MASK);
                sr += static_cast<double>(v.re);
                si += static_cast<double>(v.im);
            }
            return {static_cast<T>(sr), static_cast<T>(si)};
        }
        cplx<T> acc{T(1), T(0)};
        for (uint32_t e = e0; e < e1; ++e) {
            const uint32_t r = g.col[e];
            const uint32_t tag = r >> 30;
            if (tag == TAG_IND) {
                if (!ind_hit(r)) acc = {T(0), T(0)};
                continue;
            }
            const cplx<T> v = (tag == TAG_NODE) ? val[(r & REF_MASK) * WAVE + lane] : slot(r & REF_MASK);
            acc = cmul(acc, v);
        }
        return acc;
    }

    // product of the siblings of edge e inside parent p (1 for a sum parent)
    __device__ __forceinline__ cplx<T> sibling_product(uint32_t p, uint32_t e) const {
        cplx<T> acc{T(1), T(0)};
        if (g.op[p] == 0) return acc;
        const uint32_t e0 = g.row_ptr[p], e1 = g.row_ptr[p + 1];
        for (uint32_t f = e0; f < e1; ++f) {
            if (f == e) continue;
            const uint32_t r = g.col[f];
            if ((r >> 30) == TAG_IND) {
                if (!ind_hit(r)) acc = {T(0), T(0)};
                continue;
            }
            acc = cmul(acc, (r >> 30) == TAG_NODE ? val[(r & REF_MASK) * WAVE + lane]
                                                  : slot(r & REF_MASK));
        }
        return acc;
    }

    // upward pass over all levels (all waves of the block)
    __device__ void forward(int wave, int nwaves) {
        for (int l = 0; l < g.L; ++l) {
            const uint32_t n0 = g.level_ptr[l], n1 = g.level_ptr[l + 1];
            for (uint32_t i = n0 + wave; i < n1; i += nwaves) {
                val[i * WAVE + lane] = eval_node(i);
            }
            __syncthreads();
        }
    }

    // downward pass: adj[c] = d root / d c, pull form over parent edges
    __device__ void backward(cplx<T> *adj, int wave, int nwaves) const {
        for (int l = g.L - 1; l >= 0; --l) {
            const uint32_t n0 = g.level_ptr[l], n1 = g.level_ptr[l + 1];
            for (uint32_t c = n0 + wave; c < n1; c += nwaves) {
                double ar = 0.0, ai = 0.0;
                if (c == static_cast<uint32_t>(g.root)) {
                    ar = 1.0;
                } else {
                    const uint32_t q0 = g.par_ptr[c], q1 = g.par_ptr[c + 1];
                    for (uint32_t q = q0; q < q1; ++q) {
                        const uint32_t e = g.par_edge[q];
                        const uint32_t p = g.edge_parent[e];
                        const cplx<T> t = cmul(adj[p * WAVE + lane], sibling_product(p, e));
                        ar += static_cast<double>(t.re);
                        ai += static_cast<double>(t.im);
                    }
                }
                adj[c * WAVE + lane] = {static_cast<T>(ar), static_cast<T>(ai)};
            }
            __syncthreads();
        }
    }

    // d root / d leaf (leaf index: indicators first, then slots)
    __device__ __forceinline__ cplx<T> leaf_adjoint(const cplx<T> *adj, uint32_t li) const {
        double ar = 0.0, ai = 0.0;
        const uint32_t q0 = g.leaf_ptr[li], q1 = g.leaf_ptr[li + 1];
        for (uint32_t q = q0; q < q1; ++q) {
            const uint32_t e = g.leaf_edge[q];
            const uint32_t p = g.edge_parent[e];
            const cplx<T> t = cmul(adj[p * WAVE + lane], sibling_product(p, e));
            ar += static_cast<double>(t.re);
            ai += static_cast<double>(t.im);
        }
        return {static_cast<T>(ar), static_cast<T>(ai)};
    }
};

// Stage one tile's evidence and angle weights into LDS.
template <typename T>
__device__ void stage_tile(const DevGraph &g, uint64_t *ev_s, cplx<T> *ang_s, const uint64_t *evidence,
                           const int32_t *param_of, const double *theta, int64_t b, bool valid,
                           int lane, int wave, int nwaves) {
    for (int w = wave; w < g.W; w += nwaves) ev_s[w * WAVE + lane] = valid ? evidence[b * g.W + w] : 0ull;
    const int p = valid ? param_of[b] : 0;
    const double *trow = theta + static_cast<int64_t>(p) * g.K;
    for (int s = wave; s < g.S_ang; s += nwaves) {
        double re, im;
        slot_value(g.slots[s], trow, nullptr, re, im);
        ang_s[s * WAVE + lane] = {static_cast<T>(re), static_cast<T>(im)};
    }
}

// ---------------------------------------------------------------------------
// upward pass for a batch (amplitude queries)
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_eval(DevGraph g, const double *theta, const int32_t *param_of,
                                                const uint64_t *evidence, int64_t B, const cplx<T> *wfix,
                                                cplx<T> *vals, size_t per_wg, cplx<T> *amp_out,
                                                double *prob_out) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *ev_s = reinterpret_cast<uint64_t *>(smem);
    cplx<T> *ang_s = reinterpret_cast<cplx<T> *>(smem + static_cast<size_t>(g.W) * WAVE * 8);
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = static_cast<int>(uniform_u32(threadIdx.x / WAVE));
    const int nwaves = blockDim.x / WAVE;
    cplx<T> *val = vals + per_wg * blockIdx.x;
    const int64_t n_tiles = (B + WAVE - 1) / WAVE;
    Tile<T> t{g, val, ev_s, ang_s, wfix, lane};
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t b = tile * WAVE + lane;
        const bool valid = b < B;
        stage_tile(g, ev_s, ang_s, evidence, param_of, theta, b, valid, lane, wave, nwaves);
        __syncthreads();
        t.forward(wave, nwaves);
        if (wave == 0 && valid) {
            cplx<T> f = val[static_cast<uint32_t>(g.root) * WAVE + lane];
            amp_out[b] = f;
            if (prob_out) {
                double re = static_cast<double>(f.re), im = static_cast<double>(f.im);
                prob_out[b] = re * re + im * im;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// upward + downward pass + chain rule (gradients)
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_grad(DevGraph g, const double *theta, const int32_t *param_of,
                                                const uint64_t *evidence, int64_t B, const cplx<T> *wfix,
                                                cplx<T> *vals, size_t per_wg, int mode,
                                                const cplx<T> *cotangent, const double *weight,
                                                double *contrib, cplx<T> *amp_out,
                                                cplx<T> *dfdtheta_out, cplx<T> *dind_out) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *ev_s = reinterpret_cast<uint64_t *>(smem);
    cplx<T> *ang_s = reinterpret_cast<cplx<T> *>(smem + static_cast<size_t>(g.W) * WAVE * 8);
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = static_cast<int>(uniform_u32(threadIdx.x / WAVE));
    const int nwaves = blockDim.x / WAVE;
    cplx<T> *val = vals + per_wg * blockIdx.x;
    cplx<T> *adj = val + static_cast<size_t>(g.N) * WAVE;
    cplx<T> *dsl = adj + static_cast<size_t>(g.N) * WAVE;    // [S_ang][64]
    const int64_t n_tiles = (B + WAVE - 1) / WAVE;
    Tile<T> t{g, val, ev_s, ang_s, wfix, lane};
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t b = tile * WAVE + lane;
        const bool valid = b < B;
        stage_tile(g, ev_s, ang_s, evidence, param_of, theta, b, valid, lane, wave, nwaves);
        __syncthreads();
        t.forward(wave, nwaves);
        t.backward(adj, wave, nwaves);
        const int p = valid ? param_of[b] : 0;
        const double *trow = theta + static_cast<int64_t>(p) * g.K;
        for (int s = wave; s < g.S_ang; s += nwaves) {
            cplx<T> a = t.leaf_adjoint(adj, static_cast<uint32_t>(g.n_ind + s));
            double dre, dim;
            slot_dvalue(g.slots[s], trow, dre, dim);
            dsl[s * WAVE + lane] = cmul(a, cplx<T>{static_cast<T>(dre), static_cast<T>(dim)});
        }
        if (dind_out) {
            for (int li = wave; li < g.n_ind; li += nwaves) {
                cplx<T> a = t.leaf_adjoint(adj, static_cast<uint32_t>(li));
                if (valid) dind_out[b * g.n_ind + li] = a;
            }
        }
        __syncthreads();
        // cotangent of the root value
        const cplx<T> f = val[static_cast<uint32_t>(g.root) * WAVE + lane];
        double gre = 0.0, gim = 0.0;
        if (valid) {
            if (mode == 0) {
                gre = static_cast<double>(cotangent[b].re);
                gim = static_cast<double>(cotangent[b].im);
            } else {
                const double fr = static_cast<double>(f.re), fi = static_cast<double>(f.im);
                double scale = 2.0 * weight[b];
                if (mode == 2) {
                    const double m2 = fr * fr + fi * fi;
                    scale = m2 > 0.0 ? scale / m2 : 0.0;
                }
                gre = scale * fr;
                gim = scale * fi;
            }
        }
        for (int j = wave; j < g.K; j += nwaves) {
            double sre = 0.0, sim = 0.0;
            for (int s = 0; s < g.S_ang; ++s) {
                if (g.slots[s].index != j) continue;
                const cplx<T> d = dsl[s * WAVE + lane];
                sre += static_cast<double>(d.re);
                sim += static_cast<double>(d.im);
            }
            if (valid) {
                // Re(g * conj(df/dtheta_j))
                contrib[b * g.K + j] = gre * sre + gim * sim;
                if (dfdtheta_out) dfdtheta_out[b * g.K + j] = {static_cast<T>(sre), static_cast<T>(sim)};
            }
        }
        if (wave == 0 && valid && amp_out) amp_out[b] = f;
        __syncthreads();
    }
}

// grad[p][j] = sum over b with param_of[b] == p of contrib[b][j], fixed order.
__global__ __launch_bounds__(BLOCK) void k_grad_reduce(const int32_t *param_of, int64_t B, int K,
                                                       const double *contrib, double *grad) {
    __shared__ double red[BLOCK];
    const int p = blockIdx.x;
    for (int j = 0; j < K; ++j) {
        double acc = 0.0;
        for (int64_t b = threadIdx.x; b < B; b += BLOCK) {
            if (param_of[b] == p) acc += contrib[b * K + j];
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = BLOCK / 2; w > 0; w >>= 1) {
            if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) grad[static_cast<int64_t>(p) * K + j] = red[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Gibbs sampler
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double rng_uniform(uint64_t seed, uint64_t chain, uint64_t sweep, uint64_t var) {
    uint64_t inner = mix64((sweep << 20) ^ var);
    uint64_t top = mix64(seed ^ mix64(chain ^ inner));
    return static_cast<double>(top >> 11) * (1.0 / 9007199254740992.0);
}

constexpr uint64_t INIT_SWEEP = 0xFFFFFFFFull;


template <typename T>
__global__ __launch_bounds__(BLOCK) void k_sample(DevGraph g, const double *theta, const cplx<T> *wfix,
                                                  cplx<T> *vals, size_t per_wg, SampleArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *ev_s = reinterpret_cast<uint64_t *>(smem);
    cplx<T> *ang_s = reinterpret_cast<cplx<T> *>(smem + static_cast<size_t>(g.W) * WAVE * 8);
    __shared__ int64_t s_chain[WAVE];
    __shared__ int32_t s_pos[WAVE];
    __shared__ uint32_t s_sweep[WAVE];
    __shared__ int32_t s_emitted[WAVE];
    __shared__ int64_t s_rounds[WAVE];

    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = static_cast<int>(uniform_u32(threadIdx.x / WAVE));
    const int nwaves = blockDim.x / WAVE;
    cplx<T> *val = vals + per_wg * blockIdx.x;
    cplx<T> *adj = val + static_cast<size_t>(g.N) * WAVE;
    cplx<T> *D = adj + static_cast<size_t>(g.N) * WAVE;    // [n_ind][64]
    Tile<T> t{g, val, ev_s, ang_s, wfix, lane};
    const int64_t stride = static_cast<int64_t>(gridDim.x) * WAVE;
    const uint32_t total_sweeps = static_cast<uint32_t>(a.burn_in) +
                                  static_cast<uint32_t>(a.spc) * static_cast<uint32_t>(a.thin);
    const uint64_t xmask = g.n_qubits >= 64 ? ~0ull : ((1ull << g.n_qubits) - 1ull);

    auto init_chain = [&](int64_t ch) {
        // wave 0 only
        s_chain[lane] = ch;
        s_pos[lane] = 0;
        s_sweep[lane] = 0;
        s_emitted[lane] = 0;
        s_rounds[lane] = 0;
        for (int w = 0; w < g.W; ++w) ev_s[w * WAVE + lane] = 0ull;
        if (ch >= 0) {
            uint64_t x = 0;
            for (int q = 0; q < g.n_qubits; ++q) {
                if (rng_uniform(a.seed, static_cast<uint64_t>(ch), INIT_SWEEP, static_cast<uint64_t>(q)) < 0.5)
                    x |= (1ull << q);
            }
            ev_s[lane] = x;
        }
    };

    if (wave == 0) {
        int64_t ch = static_cast<int64_t>(blockIdx.x) * WAVE + lane;
        init_chain(ch < a.total_chains ? ch : -1);
    }
    __syncthreads();

    for (;;) {
        const int64_t ch = s_chain[lane];
        const int any = __syncthreads_or(ch >= 0 ? 1 : 0);
        if (!any) break;
        // angle weights of this lane's parameter set
        const int p = ch >= 0 ? static_cast<int>(ch / a.cpp) : 0;
        const double *trow = theta + static_cast<int64_t>(p) * g.K;
        for (int s = wave; s < g.S_ang; s += nwaves) {
            double re, im;
            slot_value(g.slots[s], trow, nullptr, re, im);
            ang_s[s * WAVE + lane] = {static_cast<T>(re), static_cast<T>(im)};
        }
        __syncthreads();
        t.forward(wave, nwaves);
        t.backward(adj, wave, nwaves);
        for (int li = wave; li < g.n_ind; li += nwaves) D[li * WAVE + lane] = t.leaf_adjoint(adj, static_cast<uint32_t>(li));
        __syncthreads();

        if (wave == 0 && ch >= 0) {
            s_rounds[lane] += 1;
            int32_t pos = s_pos[lane];
            uint32_t sweep = s_sweep[lane];
            int32_t emitted = s_emitted[lane];
            bool done = false;
            for (;;) {
                const int v = pos;
                const uint32_t fld = g.var_field[v];
                const uint32_t word = fld >> 8, shift = (fld >> 2) & 63u, width = (fld & 3u) + 1u;
                const uint64_t fmask = (1ull << width) - 1ull;
                const uint32_t cur = static_cast<uint32_t>((ev_s[word * WAVE + lane] >> shift) & fmask);
                const uint32_t base = g.ind_base[v];
                const int dom = static_cast<int>(g.ind_base[v + 1] - base);
                double w[MAX_DOM];
                double total = 0.0;
                for (int u = 0; u < dom; ++u) {
                    const cplx<T> d = D[(base + u) * WAVE + lane];
                    const double re = static_cast<double>(d.re), im = static_cast<double>(d.im);
                    w[u] = __dadd_rn(__dmul_rn(re, re), __dmul_rn(im, im));
                    total = __dadd_rn(total, w[u]);
                }
                uint32_t pick = cur;
                if (total > 0.0) {
                    const double r = rng_uniform(a.seed, static_cast<uint64_t>(ch), sweep, static_cast<uint64_t>(v));
                    const double target = __dmul_rn(r, total);
                    double acc = 0.0;
                    int last_pos = -1;
                    int chosen = -1;
                    for (int u = 0; u < dom; ++u) {
                        acc = __dadd_rn(acc, w[u]);
                        if (w[u] > 0.0) last_pos = u;
                        if (target < acc) { chosen = u; break; }
                    }
                    if (chosen < 0) chosen = last_pos;
                    if (chosen >= 0) pick = static_cast<uint32_t>(chosen);
                }
                const bool changed = pick != cur;
                if (changed) {
                    uint64_t wv = ev_s[word * WAVE + lane];
                    wv = (wv & ~(fmask << shift)) | (static_cast<uint64_t>(pick) << shift);
                    ev_s[word * WAVE + lane] = wv;
                }
                pos += 1;
                if (pos == g.n_vars) {
                    pos = 0;
                    sweep += 1;
                    if (sweep > static_cast<uint32_t>(a.burn_in) &&
                        (sweep - static_cast<uint32_t>(a.burn_in)) % static_cast<uint32_t>(a.thin) == 0u) {
                        const int64_t c_loc = ch % a.cpp;
                        const int64_t S = static_cast<int64_t>(a.cpp) * a.spc;
                        const int64_t idx = static_cast<int64_t>(p) * S + c_loc * a.spc + emitted;
                        const uint64_t x = ev_s[lane] & xmask;
                        a.samples[idx * a.nwq] = x;
                        for (int w2 = 1; w2 < a.nwq; ++w2) a.samples[idx * a.nwq + w2] = 0ull;
                        if (a.states_out) {
                            for (int w2 = 0; w2 < g.W; ++w2) a.states_out[idx * g.W + w2] = ev_s[w2 * WAVE + lane];
                        }
                        if (a.cost_out) {
                            int c = 0;
                            for (int e = 0; e < a.n_cost_edges; ++e) {
                                const int i0 = a.cost_edges[2 * e], i1 = a.cost_edges[2 * e + 1];
                                c += static_cast<int>(((x >> i0) ^ (x >> i1)) & 1ull);
                            }
                            a.cost_out[idx] = static_cast<double>(c);
                        }
                        emitted += 1;
                    }
                    if (sweep >= total_sweeps) { done = true; break; }
                }
                if (changed) break;
            }
            if (done) {
                if (a.rounds_out) a.rounds_out[ch] = s_rounds[lane];
                const int64_t nxt = ch + stride;
                init_chain(nxt < a.total_chains ? nxt : -1);
            } else {
                s_pos[lane] = pos;
                s_sweep[lane] = sweep;
                s_emitted[lane] = emitted;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// launch wrappers (called by the host runtime)
// ---------------------------------------------------------------------------

__global__ void k_fill_zero_f64(double *p, int64_t n) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(k_fill_zero_f64, dim3(static_cast<unsigned>(blocks)), dim3(threads), 0, st, p, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fixed_slots(const DevGraph &g, const double *noise, void *wfix, hipStream_t st) {
    int threads = 64;
    int blocks = (g.S + threads - 1) / threads;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fixed_slots<T>, dim3(blocks), dim3(threads), 0, st, g, noise,
                       reinterpret_cast<cplx<T> *>(wfix));
    return hipGetLastError();
}

size_t lds_bytes(const DevGraph &g, size_t csize) {
    return static_cast<size_t>(g.W) * WAVE * 8 + static_cast<size_t>(g.S_ang) * WAVE * csize;
}

template <typename T>
hipError_t launch_eval(const DevGraph &g, int grid, const double *theta, const int32_t *param_of,
                       const uint64_t *evidence, int64_t B, const void *wfix, void *vals, size_t per_wg_elems,
                       void *amp_out, double *prob_out, hipStream_t st) {
    size_t lds = lds_bytes(g, sizeof(cplx<T>));
    hipLaunchKernelGGL(k_eval<T>, dim3(grid), dim3(BLOCK), lds, st, g, theta, param_of, evidence, B,
                       reinterpret_cast<const cplx<T> *>(wfix), reinterpret_cast<cplx<T> *>(vals),
                       per_wg_elems, reinterpret_cast<cplx<T> *>(amp_out), prob_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_grad(const DevGraph &g, int grid, const double *theta, const int32_t *param_of,
                       const uint64_t *evidence, int64_t B, const void *wfix, void *vals, size_t per_wg_elems,
                       int mode, const void *cotangent, const double *weight, double *contrib, int P,
                       double *grad, void *amp_out, void *dfdtheta_out, void *dind_out, hipStream_t st) {
    size_t lds = lds_bytes(g, sizeof(cplx<T>));
    hipLaunchKernelGGL(k_grad<T>, dim3(grid), dim3(BLOCK), lds, st, g, theta, param_of, evidence, B,
                       reinterpret_cast<const cplx<T> *>(wfix), reinterpret_cast<cplx<T> *>(vals),
                       per_wg_elems, mode, reinterpret_cast<const cplx<T> *>(cotangent), weight, contrib,
                       reinterpret_cast<cplx<T> *>(amp_out), reinterpret_cast<cplx<T> *>(dfdtheta_out),
                       reinterpret_cast<cplx<T> *>(dind_out));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (g.K > 0 && P > 0) {
        hipLaunchKernelGGL(k_grad_reduce, dim3(P), dim3(BLOCK), 0, st, param_of, B, g.K, contrib, grad);
        err = hipGetLastError();
    }
    return err;
}

template <typename T>
hipError_t launch_sample(const DevGraph &g, int grid, const double *theta, const void *wfix, void *vals,
                         size_t per_wg_elems, const SampleArgs &a, hipStream_t st) {
    size_t lds = lds_bytes(g, sizeof(cplx<T>));
    hipLaunchKernelGGL(k_sample<T>, dim3(grid), dim3(BLOCK), lds, st, g, theta,
                       reinterpret_cast<const cplx<T> *>(wfix), reinterpret_cast<cplx<T> *>(vals),
                       per_wg_elems, a);
    return hipGetLastError();
}

template hipError_t launch_fixed_slots<float>(const DevGraph &, const double *, void *, hipStream_t);
template hipError_t launch_fixed_slots<double>(const DevGraph &, const double *, void *, hipStream_t);
template hipError_t launch_eval<float>(const DevGraph &, int, const double *, const int32_t *, const uint64_t *,
                                       int64_t, const void *, void *, size_t, void *, double *, hipStream_t);
template hipError_t launch_eval<double>(const DevGraph &, int, const double *, const int32_t *, const uint64_t *,
                                        int64_t, const void *, void *, size_t, void *, double *, hipStream_t);
template hipError_t launch_grad<float>(const DevGraph &, int, const double *, const int32_t *, const uint64_t *,
                                       int64_t, const void *, void *, size_t, int, const void *, const double *,
                                       double *, int, double *, void *, void *, void *, hipStream_t);
template hipError_t launch_grad<double>(const DevGraph &, int, const double *, const int32_t *, const uint64_t *,
                                        int64_t, const void *, void *, size_t, int, const void *, const double *,
                                        double *, int, double *, void *, void *, void *, hipStream_t);
template hipError_t launch_sample<float>(const DevGraph &, int, const double *, const void *, void *, size_t,
                                         const SampleArgs &, hipStream_t);
template hipError_t launch_sample<double>(const DevGraph &, int, const double *, const void *, void *, size_t,
                                          const SampleArgs &, hipStream_t);

}  // namespace qkc
