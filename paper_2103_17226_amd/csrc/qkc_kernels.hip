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
#include <hipcub/hipcub.hpp>

#include "qkc_internal.h"

namespace qkc {

template <typename T>
struct cplx {
    T re, im;
};

// Complex product with its fused multiply-adds written out, so that every
// pass rounds it the same way wherever it is inlined (contraction left to
// the compiler may pick a different fused form at different call sites).
__device__ __forceinline__ cplx<float> cmul(cplx<float> a, cplx<float> b) {
    return {__builtin_fmaf(a.re, b.re, -(a.im * b.im)), __builtin_fmaf(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ cplx<double> cmul(cplx<double> a, cplx<double> b) {
    return {__builtin_fma(a.re, b.re, -(a.im * b.im)), __builtin_fma(a.re, b.im, a.im * b.re)};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
    return {a.re + b.re, a.im + b.im};
}

// A leaf weight as the passes use it, 16 bytes for both dtypes.  complex128
// keeps it exact; complex64 keeps the FP64 weight as hi + lo, two FP32
// parts, and the upward pass multiplies by both: a weight rounded to FP32
// once and shared by hundreds of channels (one damping strength, one angle)
// would otherwise put the same relative error into every factor of a path.
template <typename T>
struct Weight;
template <>
struct Weight<double> {
    cplx<double> w;
};
template <>
struct Weight<float> {
    cplx<float> hi, lo;
};

__device__ inline void make_weight(double re, double im, Weight<double> &w) { w.w = {re, im}; }
__device__ inline void make_weight(double re, double im, Weight<float> &w) {
    const float hr = static_cast<float>(re), hi = static_cast<float>(im);
    w.hi = {hr, hi};
    w.lo = {static_cast<float>(re - static_cast<double>(hr)), static_cast<float>(im - static_cast<double>(hi))};
}
// the weight rounded to the pass dtype (what every pass but the upward one uses)
__device__ __forceinline__ cplx<double> wval(const Weight<double> &w) { return w.w; }
__device__ __forceinline__ cplx<float> wval(const Weight<float> &w) { return w.hi; }
// a * weight: exact weight, one rounding per product in the pass dtype
__device__ __forceinline__ cplx<double> wmul(cplx<double> a, const Weight<double> &w) { return cmul(a, w.w); }
__device__ __forceinline__ cplx<float> wmul(cplx<float> a, const Weight<float> &w) {
    const float re = __builtin_fmaf(a.re, w.lo.re, -a.im * w.lo.im);
    const float im = __builtin_fmaf(a.re, w.lo.im, a.im * w.lo.re);
    return {__builtin_fmaf(a.re, w.hi.re, __builtin_fmaf(-a.im, w.hi.im, re)),
            __builtin_fmaf(a.re, w.hi.im, __builtin_fmaf(a.im, w.hi.re, im))};
}
// the weight in FP64 (sum nodes accumulate in FP64)
__device__ __forceinline__ cplx<double> wsum(const Weight<double> &w) { return w.w; }
__device__ __forceinline__ cplx<double> wsum(const Weight<float> &w) {
    return {static_cast<double>(w.hi.re) + static_cast<double>(w.lo.re),
            static_cast<double>(w.hi.im) + static_cast<double>(w.lo.im)};
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}

// Load of read-only graph data through the constant address space: the
// plan and graph arrays are written once at load time and never during a
// kernel, so a wave-uniform index becomes a scalar load (scalar cache, no
// VGPRs) instead of a vector load that every lane repeats.
template <typename U>
__device__ __forceinline__ U cld(const U *p) {
    if constexpr (__is_arithmetic(U)) {
        return *(const __attribute__((address_space(4))) U *)(p);
    } else {                                   // a small struct: its dwords, then a bit cast
        static_assert(sizeof(U) % 4 == 0, "cld: struct size must be a multiple of 4 bytes");
        struct Words {
            uint32_t w[sizeof(U) / 4];
        } x;
        const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)(p);
#pragma unroll
        for (size_t i = 0; i < sizeof(U) / 4; ++i) x.w[i] = q[i];
        return __builtin_bit_cast(U, x);
    }
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
__global__ void k_fixed_slots(DevGraph g, const double *noise, Weight<T> *wfix) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.S) return;
    const double *nz = noise ? noise : g.noise_default;
    double re = 0.0, im = 0.0;
    if (s >= g.S_ang) slot_value(g.slots[s], nullptr, nz, re, im);
    Weight<T> w;
    make_weight(re, im, w);
    wfix[s] = w;
}

// ---------------------------------------------------------------------------
// tile context
// ---------------------------------------------------------------------------

// Nodes a wave takes at a time in a level of the tile kernels: up to four,
// fewer when the level is too narrow to give every wave a full batch.
__device__ __forceinline__ uint32_t batch_nodes(uint32_t width, int nwaves) {
    const uint32_t per_wave = (width + static_cast<uint32_t>(nwaves) - 1) / static_cast<uint32_t>(nwaves);
    return per_wave < 4u ? (per_wave > 0u ? per_wave : 1u) : 4u;
}

// occurrences per group of row loads in the tile kernels' downward pass on the
// sum-of-products plan (complex64)
#ifndef GRAD_SOP_KE
#define GRAD_SOP_KE 2
#endif

template <typename T>
struct Tile {
    DevGraph g;
    cplx<T> *val;                // [N][64] node values of this tile (global)
    const uint64_t *ev;          // [W][64] evidence words (LDS)
    const Weight<T> *ang;        // [S_ang][64] angle weights (LDS)
    const Weight<T> *wfix;       // [S] fixed weights (global, uniform reads)
    int lane;

    // op of node i from the dword that holds it (a scalar load; the op
    // section is padded to 256 bytes, so the dword is inside it)
    __device__ __forceinline__ uint32_t op_at(uint32_t i) const {
        return (cld(reinterpret_cast<const uint32_t *>(g.op) + (i >> 2)) >> ((i & 3u) * 8u)) & 0xffu;
    }

    __device__ __forceinline__ bool ind_hit(uint32_t r) const {
        uint32_t u = (r >> 26) & 15u;
        uint32_t width = ((r >> 24) & 3u) + 1u;
        uint32_t word = (r >> 6) & 0x3ffffu;
        uint32_t shift = r & 63u;
        uint64_t x = (ev[word * WAVE + lane] >> shift) & ((1ull << width) - 1ull);
        return x == static_cast<uint64_t>(u);
    }

    __device__ __forceinline__ Weight<T> slot(uint32_t s) const {
        if (s < static_cast<uint32_t>(g.S_ang)) return ang[s * WAVE + lane];
        return cld(wfix + s);
    }

    // selector leaf: the weight of its variable's current value
    __device__ __forceinline__ Weight<T> sel(uint32_t q) const {
        const uint32_t *rec = g.sel + static_cast<size_t>(q) * SEL_REC;
        const uint32_t fld = cld(rec);
        const uint32_t word = fld >> 8, shift = (fld >> 2) & 63u, width = (fld & 3u) + 1u;
        const uint32_t k = static_cast<uint32_t>((ev[word * WAVE + lane] >> shift) & ((1ull << width) - 1ull));
        const uint32_t s0 = cld(rec + 1), s1 = cld(rec + 2), s2 = cld(rec + 3), s3 = cld(rec + 4);
        const uint32_t s = k == 0 ? s0 : k == 1 ? s1 : k == 2 ? s2 : k == 3 ? s3 : NO_SLOT;
        if (s == NO_SLOT) return Weight<T>{};
        return cld(wfix + s);
    }

    // weight of a slot or selector leaf reference
    __device__ __forceinline__ Weight<T> weight(uint32_t r) const {
        return (r >> 30) == TAG_SEL ? sel(r & REF_MASK) : slot(r & REF_MASK);
    }

    // value of a child reference in the pass dtype (leaves computed on the fly)
    __device__ __forceinline__ cplx<T> child(uint32_t r) const {
        const uint32_t tag = r >> 30;
        if (tag == TAG_NODE) return val[(r & REF_MASK) * WAVE + lane];
        if (tag == TAG_IND) return {ind_hit(r) ? T(1) : T(0), T(0)};
        return wval(weight(r));
    }

    // Row of a node child, or row 0 (always present) for a leaf, so that a
    // group of child loads can be issued before any branch on their kind.
    __device__ __forceinline__ cplx<T> node_row(uint32_t r) const {
        const uint32_t x = (r >> 30) == TAG_NODE ? (r & REF_MASK) : 0u;
        return val[static_cast<size_t>(x) * WAVE + lane];
    }
    // node row only for node children (the reference is uniform: a scalar branch;
    // the sentinels NO_SIBLING / MULTI_SIBLING carry tag 3 and load nothing)
    __device__ __forceinline__ cplx<T> eb_guard(uint32_t r) const {
        return (r >> 30) == TAG_NODE ? val[static_cast<size_t>(r & REF_MASK) * WAVE + lane] : cplx<T>{T(0), T(0)};
    }

    // product of the siblings of edge e inside parent p (1 for a sum parent),
    // children loaded in groups like the upward pass
    __device__ __forceinline__ cplx<T> sibling_product(uint32_t p, uint32_t e) const {
        constexpr int KC = 4;
        cplx<T> acc{T(1), T(0)};
        if (op_at(p) == 0) return acc;
        const uint32_t e0 = cld(g.row_ptr + (p)), e1 = cld(g.row_ptr + (p + 1));
        for (uint32_t fb = e0; fb < e1; fb += KC) {
            uint32_t r[KC];
            cplx<T> v[KC];
#pragma unroll
            for (int j = 0; j < KC; ++j) r[j] = fb + j < e1 ? cld(g.col + (fb + j)) : IDENT_REF;
#pragma unroll
            for (int j = 0; j < KC; ++j) v[j] = eb_guard(r[j]);
#pragma unroll
            for (int j = 0; j < KC; ++j) {
                const uint32_t f = fb + static_cast<uint32_t>(j);
                if (f >= e1) break;
                if (f == e) continue;
                const uint32_t tag = r[j] >> 30;
                if (tag == TAG_IND) {
                    if (!ind_hit(r[j])) acc = {T(0), T(0)};
                    continue;
                }
                acc = cmul(acc, tag == TAG_NODE ? v[j] : child(r[j]));
            }
        }
        return acc;
    }

    // upward pass over all levels (all waves of the block).  A wave takes KB
    // consecutive nodes of a level at a time and walks their children
    // (contiguous in col) in groups of KC whose rows are loaded together;
    // each node is summed (FP64) or multiplied (pass dtype, leaf weights
    // applied at full precision by wmul) in child order and stored when its
    // last child is in.
    __device__ void forward(int wave, int nwaves) {
        constexpr int KC = 4;
        for (int l = 0; l < g.L; ++l) {
            const uint32_t n0 = cld(g.level_ptr + (l)), n1 = cld(g.level_ptr + (l + 1));
            const uint32_t kb = batch_nodes(n1 - n0, nwaves);
            for (uint32_t b0 = n0 + static_cast<uint32_t>(wave) * kb; b0 < n1;
                 b0 += static_cast<uint32_t>(nwaves) * kb) {
                const uint32_t b1 = b0 + kb < n1 ? b0 + kb : n1;
                const uint32_t e_end = cld(g.row_ptr + (b1));
                uint32_t t = b0, t_next = cld(g.row_ptr + (b0 + 1));
                bool sum = op_at(b0) == 0;
                double sr = 0.0, si = 0.0;
                cplx<T> acc{T(1), T(0)};
                for (uint32_t e = cld(g.row_ptr + (b0)); e < e_end; e += KC) {
                    uint32_t r[KC];
                    cplx<T> v[KC];
#pragma unroll
                    for (int j = 0; j < KC; ++j) r[j] = e + j < e_end ? cld(g.col + (e + j)) : IDENT_REF;
#pragma unroll
                    for (int j = 0; j < KC; ++j) v[j] = eb_guard(r[j]);
#pragma unroll
                    for (int j = 0; j < KC; ++j) {
                        const uint32_t ee = e + static_cast<uint32_t>(j);
                        if (ee >= e_end) break;
                        while (ee >= t_next) {          // node t has all its children
                            val[static_cast<size_t>(t) * WAVE + lane] =
                                sum ? cplx<T>{static_cast<T>(sr), static_cast<T>(si)} : acc;
                            sr = 0.0;
                            si = 0.0;
                            acc = {T(1), T(0)};
                            ++t;
                            t_next = cld(g.row_ptr + (t + 1));
                            sum = op_at(t) == 0;
                        }
                        const uint32_t tag = r[j] >> 30;
                        if (tag == TAG_IND) {
                            const bool hit = ind_hit(r[j]);
                            if (sum) sr += hit ? 1.0 : 0.0;
                            else if (!hit) acc = {T(0), T(0)};
                            continue;
                        }
                        if (tag == TAG_NODE) {
                            if (sum) {
                                sr += static_cast<double>(v[j].re);
                                si += static_cast<double>(v[j].im);
                            } else {
                                acc = cmul(acc, v[j]);
                            }
                        } else {
                            const Weight<T> w = weight(r[j]);
                            if (sum) {
                                const cplx<double> d = wsum(w);
                                sr += d.re;
                                si += d.im;
                            } else {
                                acc = wmul(acc, w);
                            }
                        }
                    }
                }
                val[static_cast<size_t>(t) * WAVE + lane] = sum ? cplx<T>{static_cast<T>(sr), static_cast<T>(si)} : acc;
            }
            __syncthreads();
        }
    }

    // Upward pass on the sum-of-products plan (rows only for super-nodes):
    // the same arithmetic as forward() on the DAG -- a folded product's
    // factors are multiplied in child order in the pass dtype (weights at
    // full precision by wmul), a sum adds its terms in FP64 in child order,
    // a child of a sum that is not a product is added as it is (a weight in
    // FP64) -- so the root comes out bit for bit the same.  A wave takes up to four
    // consecutive super-nodes of a level and walks their factors in groups of
    // KC whose rows are loaded together.
    // LIVE: the upward pass alone, with rows reused (frec_live, srow).
    template <bool LIVE = false>
    __device__ void forward_sop(const SopPlan &sp, int wave, int nwaves) {
        constexpr int KC = 8;
        const uint64_t *frec = LIVE ? sp.frec_live : sp.frec;
        auto row_of = [&](uint32_t t) -> size_t { return LIVE ? cld(sp.srow + t) : t; };
        for (int l = 0; l < sp.L; ++l) {
            const uint32_t n0 = cld(sp.level_ptr + l), n1 = cld(sp.level_ptr + l + 1);
            const uint32_t kb = batch_nodes(n1 - n0, nwaves);
            for (uint32_t b0 = n0 + static_cast<uint32_t>(wave) * kb; b0 < n1;
                 b0 += static_cast<uint32_t>(nwaves) * kb) {
                const uint32_t b1 = b0 + kb < n1 ? b0 + kb : n1;
                const uint32_t f_end = cld(sp.fptr + b1);
                uint32_t t = b0, t_next = cld(sp.fptr + b0 + 1);
                double sr = 0.0, si = 0.0;
                cplx<T> acc{T(1), T(0)};
                for (uint32_t f = cld(sp.fptr + b0); f < f_end; f += KC) {
                    uint64_t rec[KC];
                    cplx<T> v[KC];
#pragma unroll
                    for (int j = 0; j < KC; ++j) rec[j] = f + j < f_end ? cld(frec + f + j) : static_cast<uint64_t>(IDENT_REF);
#pragma unroll
                    for (int j = 0; j < KC; ++j) v[j] = eb_guard(static_cast<uint32_t>(rec[j]));
#pragma unroll
                    for (int j = 0; j < KC; ++j) {
                        const uint32_t ff = f + static_cast<uint32_t>(j);
                        if (ff >= f_end) break;
                        while (ff >= t_next) {          // super-node t has all its terms
                            val[row_of(t) * WAVE + lane] = cplx<T>{static_cast<T>(sr), static_cast<T>(si)};
                            sr = 0.0;
                            si = 0.0;
                            ++t;
                            t_next = cld(sp.fptr + (t + 1));
                        }
                        const uint32_t r = static_cast<uint32_t>(rec[j]);
                        const bool last = (rec[j] & SOP_LAST_OF_TERM) != 0;
                        const uint32_t tag = r >> 30;
                        if (rec[j] & SOP_DIRECT) {      // a sum's own child: added as it is
                            if (tag == TAG_IND) {
                                sr += ind_hit(r) ? 1.0 : 0.0;
                            } else if (tag == TAG_NODE) {
                                sr += static_cast<double>(v[j].re);
                                si += static_cast<double>(v[j].im);
                            } else {
                                const cplx<double> d = wsum(weight(r));
                                sr += d.re;
                                si += d.im;
                            }
                            continue;
                        }
                        if (tag == TAG_IND) {
                            if (!ind_hit(r)) acc = {T(0), T(0)};
                        } else if (tag == TAG_NODE) {
                            acc = cmul(acc, v[j]);
                        } else {
                            acc = wmul(acc, weight(r));
                        }
                        if (last) {
                            sr += static_cast<double>(acc.re);
                            si += static_cast<double>(acc.im);
                            acc = {T(1), T(0)};
                        }
                    }
                }
                val[row_of(t) * WAVE + lane] = cplx<T>{static_cast<T>(sr), static_cast<T>(si)};
            }
            __syncthreads();
        }
    }

    // Adjoint sums on the sum-of-products plan: out(t, sum over the
    // occurrences of target t of adj[parent] times its siblings) for the
    // targets [t0, t1), the occurrences (contiguous per target, in increasing
    // parent order) walked in groups of KE whose adjoint and sibling rows are
    // loaded together; terms added in FP64 in that order.  Siblings that are
    // leaves take their pass-dtype value (weights rounded, as in backward()).
    template <typename Out>
    __device__ __forceinline__ void pull_sop(const SopPlan &sp, const cplx<T> *adj, uint32_t t0, uint32_t t1,
                                             Out out) const {
        constexpr int KE = sizeof(T) == 4 ? GRAD_SOP_KE : 2;
        const uint32_t e_end = cld(sp.ostart + t1);
        uint32_t t = t0, t_next = cld(sp.ostart + t0 + 1);
        double ar = 0.0, ai = 0.0;
        for (uint32_t e = cld(sp.ostart + t0); e < e_end; e += KE) {
            uint32_t rr[KE][4];
            cplx<T> ap[KE], sv[KE][3];
#pragma unroll
            for (int j = 0; j < KE; ++j) {
                if (e + j < e_end) {
                    const uint32_t *q = sp.occ + 4 * static_cast<size_t>(e + j);
#pragma unroll
                    for (int k = 0; k < 4; ++k) rr[j][k] = cld(q + k);
                } else {
                    rr[j][0] = 0u;
                    rr[j][1] = rr[j][2] = rr[j][3] = NO_SIBLING;
                }
            }
#pragma unroll
            for (int j = 0; j < KE; ++j) {
                ap[j] = adj[static_cast<size_t>(rr[j][0]) * WAVE + lane];
#pragma unroll
                for (int k = 0; k < 3; ++k) sv[j][k] = eb_guard(rr[j][k + 1]);
            }
#pragma unroll
            for (int j = 0; j < KE; ++j) {
                const uint32_t ee = e + static_cast<uint32_t>(j);
                if (ee >= e_end) break;
                while (ee >= t_next) {
                    out(t, cplx<T>{static_cast<T>(ar), static_cast<T>(ai)});
                    ar = 0.0;
                    ai = 0.0;
                    ++t;
                    t_next = cld(sp.ostart + (t + 1));
                }
                cplx<T> term = ap[j];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const uint32_t r = rr[j][k + 1];
                    if (r != NO_SIBLING) term = cmul(term, (r >> 30) == TAG_NODE ? sv[j][k] : child(r));
                }
                ar += static_cast<double>(term.re);
                ai += static_cast<double>(term.im);
            }
        }
        for (; t < t1; ++t) {
            out(t, cplx<T>{static_cast<T>(ar), static_cast<T>(ai)});
            ar = 0.0;
            ai = 0.0;
        }
    }

    // downward pass on the sum-of-products plan: adj[s] = d root / d s for
    // every super-node, level by level from the root
    __device__ void backward_sop(const SopPlan &sp, cplx<T> *adj, int wave, int nwaves) const {
        const uint32_t root = static_cast<uint32_t>(sp.root);
        for (int l = sp.L - 1; l >= 0; --l) {
            const uint32_t n0 = cld(sp.level_ptr + l), n1 = cld(sp.level_ptr + l + 1);
            const uint32_t kb = batch_nodes(n1 - n0, nwaves);
            for (uint32_t b0 = n0 + static_cast<uint32_t>(wave) * kb; b0 < n1;
                 b0 += static_cast<uint32_t>(nwaves) * kb) {
                const uint32_t b1 = b0 + kb < n1 ? b0 + kb : n1;
                pull_sop(sp, adj, b0, b1, [&](uint32_t i, cplx<T> v) {
                    adj[static_cast<size_t>(i) * WAVE + lane] = i == root ? cplx<T>{T(1), T(0)} : v;
                });
            }
            __syncthreads();
        }
    }

    // d root / d (angle slot s) on the sum-of-products plan
    __device__ __forceinline__ cplx<T> slot_adjoint_sop(const SopPlan &sp, const cplx<T> *adj, uint32_t s) const {
        const uint32_t t = static_cast<uint32_t>(sp.S + g.n_ind + g.n_sel) + s;
        cplx<T> res{T(0), T(0)};
        pull_sop(sp, adj, t, t + 1, [&](uint32_t, cplx<T> v) { res = v; });
        return res;
    }

    // d root / d lambda_{v=u} on the sum-of-products plan, written to
    // out[(base + u) * ostride] (indicator leaves plus selector leaves)
    __device__ void ind_derivatives_sop(const SopPlan &sp, const cplx<T> *adj, int v, cplx<T> *out,
                                        size_t ostride) const {
        const uint32_t M = static_cast<uint32_t>(sp.S);
        const uint32_t base = cld(g.ind_base + (v)), dom = cld(g.ind_base + (v + 1)) - base;
        pull_sop(sp, adj, M + base, M + base + dom, [&](uint32_t i, cplx<T> val) { out[(i - M) * ostride] = val; });
        const uint32_t q1 = cld(g.vsel_ptr + (v + 1));
        for (uint32_t qq = cld(g.vsel_ptr + (v)); qq < q1; ++qq) {
            const uint32_t q = cld(g.vsel + (qq));
            const uint32_t tq = M + static_cast<uint32_t>(g.n_ind) + qq;
            cplx<T> A{T(0), T(0)};
            pull_sop(sp, adj, tq, tq + 1, [&](uint32_t, cplx<T> val) { A = val; });
            const uint32_t *rec = g.sel + static_cast<size_t>(q) * SEL_REC;
            for (uint32_t u = 0; u < dom && u < static_cast<uint32_t>(SEL_DOM); ++u) {
                const uint32_t sl = cld(rec + 1 + u);
                if (sl == NO_SLOT) continue;
                const cplx<T> t = cmul(A, wval(cld(wfix + sl)));
                cplx<T> &o = out[(base + u) * ostride];
                o = cadd(o, t);
            }
        }
    }

    // adj[parent] * (product of the other children) summed in FP64 over the
    // parent edges q0..q1 of a node or leaf.  recs holds one record per edge
    // (parent | sibling << 32, see DevGraph), so a group of KQ edges needs one
    // round of scalar loads before the parents' adjoint rows and the sibling
    // rows of the whole group are loaded together.  Edges whose parent has
    // three or more children take the general sibling product after the
    // group.  The order of the terms is fixed, so the result is reproducible.
    __device__ __forceinline__ cplx<T> pull_parents(const cplx<T> *adj, const uint64_t *recs, const uint32_t *edges,
                                                   uint32_t q0, uint32_t q1) const {
        constexpr int KQ = 4;
        double ar = 0.0, ai = 0.0;
        for (uint32_t qb = q0; qb < q1; qb += KQ) {
            uint64_t rr[KQ];
            cplx<T> a[KQ], sv[KQ];
#pragma unroll
            for (int j = 0; j < KQ; ++j)
                rr[j] = qb + j < q1 ? cld(recs + qb + j) : (static_cast<uint64_t>(NO_SIBLING) << 32);
#pragma unroll
            for (int j = 0; j < KQ; ++j) {
                a[j] = adj[static_cast<size_t>(static_cast<uint32_t>(rr[j])) * WAVE + lane];
                sv[j] = eb_guard(static_cast<uint32_t>(rr[j] >> 32));
            }
#pragma unroll
            for (int j = 0; j < KQ; ++j) {
                const uint32_t sib = static_cast<uint32_t>(rr[j] >> 32);
                if (qb + j >= q1 || sib == MULTI_SIBLING) continue;
                cplx<T> t = a[j];
                if (sib != NO_SIBLING) t = cmul(t, (sib >> 30) == TAG_NODE ? sv[j] : child(sib));
                ar += static_cast<double>(t.re);
                ai += static_cast<double>(t.im);
            }
            const uint32_t qe = qb + KQ < q1 ? qb + KQ : q1;
#pragma unroll 1
            for (uint32_t q = qb; q < qe; ++q) {       // parents with three or more children
                const uint64_t r = cld(recs + q);
                if (static_cast<uint32_t>(r >> 32) != MULTI_SIBLING) continue;
                const uint32_t pq = static_cast<uint32_t>(r);
                const cplx<T> t = cmul(adj[static_cast<size_t>(pq) * WAVE + lane], sibling_product(pq, cld(edges + q)));
                ar += static_cast<double>(t.re);
                ai += static_cast<double>(t.im);
            }
        }
        return {static_cast<T>(ar), static_cast<T>(ai)};
    }

    // downward pass: adj[c] = d root / d c, pull form over parent edges.  A
    // wave takes KB consecutive nodes of a level at a time and walks their
    // parent edges (contiguous in par_rec) in groups of KE whose adjoint and
    // sibling rows are loaded together; each node's terms are added in FP64
    // in edge order and its adjoint is stored once its last edge is in.
    // Edges from products of three or more children (rare) are added to the
    // stored adjoints afterwards by the same wave.
    __device__ void backward(cplx<T> *adj, int wave, int nwaves) const {
        constexpr int KE = sizeof(T) == 4 ? 8 : 4;
        const uint32_t root = static_cast<uint32_t>(g.root);
        for (int l = g.L - 1; l >= 0; --l) {
            const uint32_t n0 = cld(g.level_ptr + (l)), n1 = cld(g.level_ptr + (l + 1));
            const uint32_t kb = batch_nodes(n1 - n0, nwaves);
            for (uint32_t b0 = n0 + static_cast<uint32_t>(wave) * kb; b0 < n1;
                 b0 += static_cast<uint32_t>(nwaves) * kb) {
                const uint32_t b1 = b0 + kb < n1 ? b0 + kb : n1;
                const uint32_t e_begin = cld(g.par_ptr + (b0)), e_end = cld(g.par_ptr + (b1));
                uint32_t t = b0, t_next = cld(g.par_ptr + (b0 + 1));
                double ar = 0.0, ai = 0.0;
                bool multi = false;
                for (uint32_t e = e_begin; e < e_end; e += KE) {
                    uint64_t rr[KE];
                    cplx<T> a[KE], sv[KE];
#pragma unroll
                    for (int j = 0; j < KE; ++j)
                        rr[j] = e + j < e_end ? cld(g.par_rec + (e + j)) : (static_cast<uint64_t>(NO_SIBLING) << 32);
#pragma unroll
                    for (int j = 0; j < KE; ++j) {
                        a[j] = adj[static_cast<size_t>(static_cast<uint32_t>(rr[j])) * WAVE + lane];
                        sv[j] = eb_guard(static_cast<uint32_t>(rr[j] >> 32));
                    }
#pragma unroll
                    for (int j = 0; j < KE; ++j) {
                        const uint32_t ee = e + static_cast<uint32_t>(j);
                        if (ee >= e_end) break;
                        while (ee >= t_next) {
                            adj[static_cast<size_t>(t) * WAVE + lane] =
                                t == root ? cplx<T>{T(1), T(0)} : cplx<T>{static_cast<T>(ar), static_cast<T>(ai)};
                            ar = 0.0;
                            ai = 0.0;
                            ++t;
                            t_next = cld(g.par_ptr + (t + 1));
                        }
                        const uint32_t sib = static_cast<uint32_t>(rr[j] >> 32);
                        if (sib == MULTI_SIBLING) {
                            multi = true;
                            continue;
                        }
                        cplx<T> term = a[j];
                        if (sib != NO_SIBLING) term = cmul(term, (sib >> 30) == TAG_NODE ? sv[j] : child(sib));
                        ar += static_cast<double>(term.re);
                        ai += static_cast<double>(term.im);
                    }
                }
                for (; t < b1; ++t) {
                    adj[static_cast<size_t>(t) * WAVE + lane] =
                        t == root ? cplx<T>{T(1), T(0)} : cplx<T>{static_cast<T>(ar), static_cast<T>(ai)};
                    ar = 0.0;
                    ai = 0.0;
                }
                if (multi) {
#pragma unroll 1
                    for (uint32_t c = b0; c < b1; ++c) {
                        const uint32_t q1 = cld(g.par_ptr + (c + 1));
                        double mr = 0.0, mi = 0.0;
                        bool any = false;
#pragma unroll 1
                        for (uint32_t q = cld(g.par_ptr + (c)); q < q1; ++q) {
                            const uint64_t r = cld(g.par_rec + (q));
                            if (static_cast<uint32_t>(r >> 32) != MULTI_SIBLING) continue;
                            const uint32_t pq = static_cast<uint32_t>(r);
                            const cplx<T> tm = cmul(adj[static_cast<size_t>(pq) * WAVE + lane], sibling_product(pq, cld(g.par_edge + (q))));
                            mr += static_cast<double>(tm.re);
                            mi += static_cast<double>(tm.im);
                            any = true;
                        }
                        if (any) {
                            cplx<T> &o = adj[static_cast<size_t>(c) * WAVE + lane];
                            o = {static_cast<T>(static_cast<double>(o.re) + mr), static_cast<T>(static_cast<double>(o.im) + mi)};
                        }
                    }
                }
            }
            __syncthreads();
        }
    }

    // d root / d lambda_{v=u} for every value u of variable v, written to
    // out[(base + u) * ostride] (indicator leaves plus selector leaves)
    __device__ void ind_derivatives(const cplx<T> *adj, int v, cplx<T> *out, size_t ostride) const {
        const uint32_t base = cld(g.ind_base + (v)), dom = cld(g.ind_base + (v + 1)) - base;
        for (uint32_t u = 0; u < dom; ++u) out[(base + u) * ostride] = leaf_adjoint(adj, base + u);
        const uint32_t q1 = cld(g.vsel_ptr + (v + 1));
        for (uint32_t qq = cld(g.vsel_ptr + (v)); qq < q1; ++qq) {
            const uint32_t q = cld(g.vsel + (qq));
            const cplx<T> A = leaf_adjoint(adj, static_cast<uint32_t>(g.n_ind + g.S) + q);
            const uint32_t *rec = g.sel + static_cast<size_t>(q) * SEL_REC;
            for (uint32_t u = 0; u < dom && u < static_cast<uint32_t>(SEL_DOM); ++u) {
                const uint32_t sl = cld(rec + 1 + u);
                if (sl == NO_SLOT) continue;
                const cplx<T> t = cmul(A, wval(cld(wfix + sl)));
                cplx<T> &o = out[(base + u) * ostride];
                o = cadd(o, t);
            }
        }
    }

    // d root / d leaf (leaf index: indicators first, then slots)
    __device__ __forceinline__ cplx<T> leaf_adjoint(const cplx<T> *adj, uint32_t li) const {
        return pull_parents(adj, g.leaf_rec, g.leaf_edge, cld(g.leaf_ptr + (li)), cld(g.leaf_ptr + (li + 1)));
    }
};

// Stage one tile's evidence and angle weights into LDS.
template <typename T>
__device__ bool stage_tile(const DevGraph &g, uint64_t *ev_s, Weight<T> *ang_s, const uint64_t *evidence,
                           const int32_t *param_of, int P, const double *theta, int64_t b, bool valid,
                           int lane, int wave, int nwaves) {
    for (int w = wave; w < g.W; w += nwaves) ev_s[w * WAVE + lane] = valid ? evidence[b * g.W + w] : 0ull;
    int p = valid ? param_of[b] : 0;
    const bool in_range = p >= 0 && p < P;       // an index outside [0, P) reads no parameters
    if (!in_range) p = 0;
    const double *trow = theta + static_cast<int64_t>(p) * g.K;
    for (int s = wave; s < g.S_ang; s += nwaves) {
        double re, im;
        slot_value(g.slots[s], trow, nullptr, re, im);
        make_weight(re, im, ang_s[s * WAVE + lane]);
    }
    return in_range;
}

// ---------------------------------------------------------------------------
// upward pass for a batch (amplitude queries)
// ---------------------------------------------------------------------------

// complex64: 8 waves per SIMD (64 VGPRs, a few spilled): rows wait on HBM and
// more resident waves hide it (16-qubit noisy QAOA, 262,144 amplitudes, on
// the binary-node plan: 6 waves 74 ms, 8 waves 66 ms)
template <typename T, bool SOP>
__global__ __launch_bounds__(MAX_BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 1, 8))) void k_eval(DevGraph g, SopPlan sp, const double *theta, const int32_t *param_of, int P,
                                                const uint64_t *evidence, int64_t B, const Weight<T> *wfix,
                                                cplx<T> *vals, size_t per_wg, cplx<T> *amp_out,
                                                double *prob_out) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *ev_s = reinterpret_cast<uint64_t *>(smem);
    Weight<T> *ang_s = reinterpret_cast<Weight<T> *>(smem + static_cast<size_t>(g.W) * WAVE * 8);
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = static_cast<int>(uniform_u32(threadIdx.x / WAVE));
    const int nwaves = blockDim.x / WAVE;
    cplx<T> *val = vals + per_wg * blockIdx.x;
    const int64_t n_tiles = (B + WAVE - 1) / WAVE;
    Tile<T> t{g, val, ev_s, ang_s, wfix, lane};
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t b = tile * WAVE + lane;
        const bool valid = b < B;
        const bool in_range = stage_tile(g, ev_s, ang_s, evidence, param_of, P, theta, b, valid, lane, wave, nwaves);
        __syncthreads();
        if constexpr (SOP) t.template forward_sop<true>(sp, wave, nwaves);
        else t.forward(wave, nwaves);
        if (wave == 0 && valid) {
            uint32_t root_row = static_cast<uint32_t>(g.root);
            if constexpr (SOP) root_row = cld(sp.srow + sp.root);
            cplx<T> f = val[static_cast<size_t>(root_row) * WAVE + lane];
            if (!in_range) f = {T(NAN), T(NAN)};
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
// most probable explanation of an outcome: max-product over the noise events
// ---------------------------------------------------------------------------
//
// On an AC whose noise-event decisions all lie above the sums over hidden
// qubit values (events decided first by the compiler), the nodes split in
// two domains.  A node with no event indicator below it holds its complex
// value as in the upward pass.  Every other node holds
//   M(n) = max over the events below n of |value(n)|^2,
// a real error probability where the maximum is defined: a product
// multiplies its children's M (a complex child or leaf contributes |v|^2;
// the events below a product's children are disjoint), a sum decides one
// variable and takes its largest branch.  Event indicators are 1 (the
// events are free); output indicators follow the evidence.  A top-down pass
// then walks, per element, from the root through the largest branch of
// every selected sum (the first in child order on ties) and every child of
// every selected product, and records each event indicator it passes: the
// events k* with |f(x, k*)|^2 = M(root).  Rows [N][64] complex128: value, or
// (M, selected flag).

__device__ __forceinline__ bool event_ref(uint32_t r, int n_qubits) {
    const uint32_t word = (r >> 6) & 0x3ffffu, shift = r & 63u;
    return word * 64u + shift >= static_cast<uint32_t>(n_qubits);
}

// max-domain quantity of a child reference: M of a max-domain node, |v|^2 of
// a complex node or weight, 1 for an event indicator, 0/1 from the evidence
// for an output indicator
__device__ __forceinline__ double mpe_child(const Tile<double> &t, const MpePlan &mp, uint32_t r) {
    const uint32_t tag = r >> 30;
    if (tag == TAG_NODE) {
        const uint32_t c = r & REF_MASK;
        const cplx<double> v = t.val[static_cast<size_t>(c) * WAVE + t.lane];
        return mp.big[c] ? v.re : __dadd_rn(__dmul_rn(v.re, v.re), __dmul_rn(v.im, v.im));
    }
    if (tag == TAG_IND) return event_ref(r, mp.n_qubits) ? 1.0 : (t.ind_hit(r) ? 1.0 : 0.0);
    const cplx<double> w = wval(t.weight(r));
    return __dadd_rn(__dmul_rn(w.re, w.re), __dmul_rn(w.im, w.im));
}

// 8 waves per SIMD (64 VGPRs, a few spilled): two 16-wave workgroups per CU
__global__ __launch_bounds__(MAX_BLOCK) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_mpe(DevGraph g, MpePlan mp, const double *theta, const int32_t *param_of,
                                               int P, const uint64_t *evidence, int64_t B,
                                               const Weight<double> *wfix, cplx<double> *vals, size_t per_wg,
                                               double *prob_out, uint64_t *mpe_out) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *ev_s = reinterpret_cast<uint64_t *>(smem);
    Weight<double> *ang_s = reinterpret_cast<Weight<double> *>(smem + static_cast<size_t>(g.W) * WAVE * 8);
    unsigned long long *k_s = reinterpret_cast<unsigned long long *>(
        smem + static_cast<size_t>(g.W) * WAVE * 8 + static_cast<size_t>(g.S_ang) * WAVE * sizeof(Weight<double>));
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = static_cast<int>(uniform_u32(threadIdx.x / WAVE));
    const int nwaves = blockDim.x / WAVE;
    cplx<double> *val = vals + per_wg * blockIdx.x;
    Tile<double> t{g, val, ev_s, ang_s, wfix, lane};
    const int64_t n_tiles = (B + WAVE - 1) / WAVE;
    const uint32_t root = static_cast<uint32_t>(g.root);
    const bool root_big = mp.big[root] != 0;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t b = tile * WAVE + lane;
        const bool valid = b < B;
        const bool in_range = stage_tile(g, ev_s, ang_s, evidence, param_of, P, theta, b, valid, lane, wave, nwaves);
        for (int w = wave; w < g.W; w += nwaves)
            k_s[w * WAVE + lane] = (valid ? evidence[b * g.W + w] : 0ull) & ~mp.event_mask[w];
        __syncthreads();
        for (int l = 0; l < g.L; ++l) {
            const uint32_t n0 = g.level_ptr[l], n1 = g.level_ptr[l + 1];
            for (uint32_t i = n0 + static_cast<uint32_t>(wave); i < n1; i += static_cast<uint32_t>(nwaves)) {
                const uint32_t e0 = g.row_ptr[i], e1 = g.row_ptr[i + 1];
                const bool sum = t.op_at(i) == 0;
                if (!mp.big[i]) {
                    cplx<double> acc = sum ? cplx<double>{0.0, 0.0} : cplx<double>{1.0, 0.0};
                    for (uint32_t e = e0; e < e1; ++e) {
                        const cplx<double> v = t.child(g.col[e]);
                        acc = sum ? cadd(acc, v) : cmul(acc, v);
                    }
                    val[static_cast<size_t>(i) * WAVE + lane] = acc;
                } else {
                    double m = sum ? 0.0 : 1.0;
                    for (uint32_t e = e0; e < e1; ++e) {
                        const double c = mpe_child(t, mp, g.col[e]);
                        m = sum ? (c > m ? c : m) : __dmul_rn(m, c);
                    }
                    val[static_cast<size_t>(i) * WAVE + lane] = {m, 0.0};
                }
            }
            __syncthreads();
        }
        if (root_big) {
            if (wave == 0) val[static_cast<size_t>(root) * WAVE + lane].im = 1.0;
            __syncthreads();
            for (int l = g.L - 1; l >= 0; --l) {
                const uint32_t n0 = g.level_ptr[l], n1 = g.level_ptr[l + 1];
                for (uint32_t i = n0 + static_cast<uint32_t>(wave); i < n1; i += static_cast<uint32_t>(nwaves)) {
                    if (!mp.big[i]) continue;
                    const bool chosen = val[static_cast<size_t>(i) * WAVE + lane].im != 0.0;
                    const uint32_t e0 = g.row_ptr[i], e1 = g.row_ptr[i + 1];
                    uint32_t lo = e0, hi = e1;
                    if (t.op_at(i) == 0) {               // the first largest branch
                        double best = -1.0;
                        for (uint32_t e = e0; e < e1; ++e) {
                            const double c = mpe_child(t, mp, g.col[e]);
                            if (c > best) {
                                best = c;
                                lo = e;
                            }
                        }
                        hi = lo + 1;
                    }
                    if (!chosen) continue;
                    for (uint32_t e = lo; e < hi; ++e) {
                        const uint32_t r = g.col[e], tag = r >> 30;
                        if (tag == TAG_NODE) {
                            const uint32_t c = r & REF_MASK;
                            if (mp.big[c]) val[static_cast<size_t>(c) * WAVE + lane].im = 1.0;
                        } else if (tag == TAG_IND && event_ref(r, mp.n_qubits)) {
                            const uint32_t u = (r >> 26) & 15u, word = (r >> 6) & 0x3ffffu, shift = r & 63u;
                            atomicOr(&k_s[word * WAVE + lane], static_cast<unsigned long long>(u) << shift);
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (valid) {
            for (int w = wave; w < g.W; w += nwaves) mpe_out[b * g.W + w] = k_s[w * WAVE + lane];
            if (wave == 0) {
                const cplx<double> v = val[static_cast<size_t>(root) * WAVE + lane];
                double m = root_big ? v.re : __dadd_rn(__dmul_rn(v.re, v.re), __dmul_rn(v.im, v.im));
                prob_out[b] = in_range ? m : static_cast<double>(NAN);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// upward + downward pass + chain rule (gradients)
// ---------------------------------------------------------------------------

// complex64: 6 waves per SIMD (80 VGPRs, a few spilled; 5 waves unbounded):
// 16-qubit noisy QAOA gradients over 262,144 elements, on the binary-node
// plan, 283 -> 255 ms
template <typename T, bool SOP>
__global__ __launch_bounds__(MAX_BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1, 8))) void k_grad(DevGraph g, SopPlan sp, const double *theta, const int32_t *param_of, int P,
                                                const uint64_t *evidence, int64_t B, const Weight<T> *wfix,
                                                cplx<T> *vals, size_t per_wg, int mode,
                                                const cplx<T> *cotangent, const double *weight,
                                                double *contrib, cplx<T> *amp_out,
                                                cplx<T> *dfdtheta_out, cplx<T> *dind_out) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *ev_s = reinterpret_cast<uint64_t *>(smem);
    Weight<T> *ang_s = reinterpret_cast<Weight<T> *>(smem + static_cast<size_t>(g.W) * WAVE * 8);
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = static_cast<int>(uniform_u32(threadIdx.x / WAVE));
    const int nwaves = blockDim.x / WAVE;
    cplx<T> *val = vals + per_wg * blockIdx.x;
    constexpr bool sop = SOP;                        // sum-of-products plan, else the DAG itself
    const size_t rows = sop ? static_cast<size_t>(sp.S) : static_cast<size_t>(g.N);
    cplx<T> *adj = val + rows * WAVE;
    cplx<T> *dsl = adj + rows * WAVE;                // [S_ang][64]
    const int64_t n_tiles = (B + WAVE - 1) / WAVE;
    Tile<T> t{g, val, ev_s, ang_s, wfix, lane};
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t b = tile * WAVE + lane;
        const bool in_batch = b < B;
        const bool in_range = stage_tile(g, ev_s, ang_s, evidence, param_of, P, theta, b, in_batch, lane, wave, nwaves);
        const bool valid = in_batch && in_range;
        __syncthreads();
        if constexpr (sop) {
            t.forward_sop(sp, wave, nwaves);
            t.backward_sop(sp, adj, wave, nwaves);
        } else {
            t.forward(wave, nwaves);
            t.backward(adj, wave, nwaves);
        }
        const int p = valid ? param_of[b] : 0;
        const double *trow = theta + static_cast<int64_t>(p) * g.K;
        for (int s = wave; s < g.S_ang; s += nwaves) {
            cplx<T> a;
            if constexpr (sop) a = t.slot_adjoint_sop(sp, adj, static_cast<uint32_t>(s));
            else a = t.leaf_adjoint(adj, static_cast<uint32_t>(g.n_ind + s));
            double dre, dim;
            slot_dvalue(g.slots[s], trow, dre, dim);
            dsl[s * WAVE + lane] = cmul(a, cplx<T>{static_cast<T>(dre), static_cast<T>(dim)});
        }
        if (dind_out) {
            // [n_ind][64] rows after the angle-weight rows of this tile's buffer
            cplx<T> *Dt = dsl + static_cast<size_t>(g.S_ang) * WAVE;
            for (int v = wave; v < g.n_vars; v += nwaves) {
                if constexpr (sop) t.ind_derivatives_sop(sp, adj, v, Dt + lane, WAVE);
                else t.ind_derivatives(adj, v, Dt + lane, WAVE);
            }
            __syncthreads();
            if (valid)
                for (int li = 0; li < g.n_ind; ++li) dind_out[b * g.n_ind + li] = Dt[static_cast<size_t>(li) * WAVE + lane];
        }
        __syncthreads();
        // cotangent of the root value
        const cplx<T> f = val[static_cast<uint32_t>(sop ? sp.root : g.root) * WAVE + lane];
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
            } else if (in_batch && dfdtheta_out) {
                dfdtheta_out[b * g.K + j] = {T(NAN), T(NAN)};
            }
        }
        if (wave == 0 && in_batch && amp_out) amp_out[b] = valid ? f : cplx<T>{T(NAN), T(NAN)};
        __syncthreads();
    }
}

// grad[p][j] = sum over b with param_of[b] == p of contrib[b][j], in an
// order fixed by the elements' relative positions: the batch indices are
// stably sorted by parameter set (a device radix sort on keys param_of, with
// out-of-range entries in an extra bucket P that is never summed), so each
// set's elements form one segment in their original order; thread t of the
// set's workgroup adds segment positions t, t + 256, ... and the 256 partial
// sums meet in a fixed tree.  O(B K) work, bit for bit the same for any
// placement of a request's rows in a larger batch.
__global__ void k_grad_keys(const int32_t *param_of, int64_t B, int P, uint32_t *keys, uint32_t *idx) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int32_t p = param_of[b];
    keys[b] = p >= 0 && p < P ? static_cast<uint32_t>(p) : static_cast<uint32_t>(P);
    idx[b] = static_cast<uint32_t>(b);
}

__device__ __forceinline__ int64_t lower_bound_u32(const uint32_t *a, int64_t n, uint32_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(BLOCK) void k_grad_segments(const uint32_t *keys, const uint32_t *idx, int64_t B, int K,
                                                         const double *contrib, double *grad) {
    __shared__ double red[BLOCK];
    const uint32_t p = blockIdx.x;
    const int64_t lo = lower_bound_u32(keys, B, p), hi = lower_bound_u32(keys, B, p + 1);
    for (int j = 0; j < K; ++j) {
        double acc = 0.0;
        for (int64_t q = lo + threadIdx.x; q < hi; q += BLOCK) acc += contrib[static_cast<int64_t>(idx[q]) * K + j];
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

// MaxCut cost of an output word over the caller's edge list: the number of
// edges whose ends differ; NaN if an edge names a qubit outside [0, n).
__device__ inline double maxcut_cost(const SampleArgs &a, uint64_t x, int n) {
    int cst = 0;
    bool bad = false;
    for (int e = 0; e < a.n_cost_edges; ++e) {
        const int i0 = a.cost_edges[2 * e], i1 = a.cost_edges[2 * e + 1];
        if (i0 < 0 || i0 >= n || i1 < 0 || i1 >= n) {
            bad = true;
            continue;
        }
        cst += static_cast<int>(((x >> i0) ^ (x >> i1)) & 1ull);
    }
    return bad ? static_cast<double>(NAN) : static_cast<double>(cst);
}


template <typename T>
__global__ __launch_bounds__(BLOCK) void k_sample(DevGraph g, const double *theta, const Weight<T> *wfix,
                                                  cplx<T> *vals, size_t per_wg, SampleArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *ev_s = reinterpret_cast<uint64_t *>(smem);
    Weight<T> *ang_s = reinterpret_cast<Weight<T> *>(smem + static_cast<size_t>(g.W) * WAVE * 8);
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
        s_pos[lane] = a.first_var;
        s_sweep[lane] = 0;
        s_emitted[lane] = 0;
        s_rounds[lane] = 0;
        for (int w = 0; w < g.W; ++w)
            ev_s[w * WAVE + lane] = (ch >= 0 && a.init_states) ? a.init_states[ch * g.W + w] : 0ull;
        if (ch >= 0 && !a.init_states) {
            uint64_t x = 0;
            for (int q = 0; q < g.n_qubits; ++q) {
                if (rng_uniform(a.seed, a.chain_offset + static_cast<uint64_t>(ch), INIT_SWEEP, static_cast<uint64_t>(q)) < 0.5)
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
            make_weight(re, im, ang_s[s * WAVE + lane]);
        }
        __syncthreads();
        t.forward(wave, nwaves);
        t.backward(adj, wave, nwaves);
        for (int v = wave; v < g.n_vars; v += nwaves) t.ind_derivatives(adj, v, D + lane, WAVE);
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
                    const double r = rng_uniform(a.seed, a.chain_offset + static_cast<uint64_t>(ch), a.first_sweep + sweep, static_cast<uint64_t>(v));
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
                    pos = a.first_var;
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
                        if (a.cost_out) a.cost_out[idx] = maxcut_cost(a, x, g.n_qubits);
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
// Gibbs sampler, streaming variant on the binary plan
// ---------------------------------------------------------------------------
//
// Lane = chain, 64 chains per workgroup of 4 waves; node values and adjoints
// live in a per-workgroup global buffer [node][64] (one coalesced row per
// node).  Each wave takes a batch of KB nodes of a level at a time: it loads
// their records with uniform (scalar) loads, issues every child-value load
// of the batch, and only then computes and stores, so that KB rows per wave
// are in flight instead of one.
//
// Every lane reads only the column it wrote itself (lane = chain), so a
// workgroup of one wavefront needs no barrier between levels: the wave's own
// stores and loads of one address stay in program order, and the next level's
// loads can issue while this level's stores drain.  With several waves per
// tile a level's rows come from other waves and the barrier is required.

__device__ __forceinline__ void level_sync(int nwaves) {
    if (nwaves > 1) __syncthreads();
}

// Rows of a workgroup's [rows][64] region through a buffer resource: the row
// offset (row x 64 x element bytes) is wave-uniform and goes in the scalar
// offset, the lane offset is one VGPR shared by every access, so a batch of
// row loads holds no 64-bit addresses in VGPRs.  The region is below 2 GiB
// (checked at launch).
template <typename T>
struct RowBuf {
    __amdgpu_buffer_rsrc_t rs;
    uint32_t lane_off;

    static constexpr uint32_t ROW_BYTES = WAVE * sizeof(cplx<T>);

    __device__ __forceinline__ RowBuf(cplx<T> *region, size_t rows, int lane)
        : rs(__builtin_amdgcn_make_buffer_rsrc(region, 0, static_cast<int>(rows * ROW_BYTES), 0x00020000)),
          lane_off(static_cast<uint32_t>(lane) * static_cast<uint32_t>(sizeof(cplx<T>))) {}

    __device__ __forceinline__ cplx<T> ld(uint32_t row) const {
        if constexpr (sizeof(T) == 4)
            return __builtin_bit_cast(cplx<T>, __builtin_amdgcn_raw_buffer_load_b64(rs, lane_off, row * ROW_BYTES, 0));
        else
            return __builtin_bit_cast(cplx<T>, __builtin_amdgcn_raw_buffer_load_b128(rs, lane_off, row * ROW_BYTES, 0));
    }
    __device__ __forceinline__ void st(uint32_t row, cplx<T> v) const {
        if constexpr (sizeof(T) == 4)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) uint32_t, v), rs,
                                                  lane_off, row * ROW_BYTES, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) uint32_t, v), rs,
                                                   lane_off, row * ROW_BYTES, 0);
    }
};

// One Gibbs visit of a variable with at most SEL_DOM values: weights w_u =
// |d root / d lambda_{v=u}|^2 in FP64, the smallest u with r * total <
// w_0 + ... + w_u, or the last value of positive weight when rounding leaves
// none; zero total keeps the current value.  The scan's own per-visit code
// performs the same operations in the same order.
__device__ __forceinline__ uint32_t gibbs_choice(const double (&w)[SEL_DOM], int dom, uint32_t cur, double r) {
    double total = 0.0;
#pragma unroll
    for (int u = 0; u < SEL_DOM; ++u)
        if (u < dom) total = __dadd_rn(total, w[u]);
    if (!(total > 0.0)) return cur;
    const double target = __dmul_rn(r, total);
    double acc = 0.0;
    int last_pos = -1, chosen = -1;
#pragma unroll
    for (int u = 0; u < SEL_DOM; ++u) {
        if (u >= dom || chosen >= 0) continue;
        acc = __dadd_rn(acc, w[u]);
        if (w[u] > 0.0) last_pos = u;
        if (target < acc) chosen = u;
    }
    if (chosen < 0) chosen = last_pos;
    return chosen >= 0 ? static_cast<uint32_t>(chosen) : cur;
}

template <typename T>
__device__ __forceinline__ double gibbs_weight(const cplx<T> &d) {
    const double re = static_cast<double>(d.re), im = static_cast<double>(d.im);
    return __dadd_rn(__dmul_rn(re, re), __dmul_rn(im, im));
}

// Batch sizes of the streaming passes on the sum-of-products plan
// (complex64; complex128 halves the factor and occurrence groups):
// super-nodes per wave batch, factors per group of row loads (upward pass),
// occurrences per group (downward pass, leaf step).
#ifndef SOP_KB
#define SOP_KB 4
#endif
#ifndef SOP_KF
#define SOP_KF 8
#endif
#ifndef SOP_KE
#define SOP_KE 4
#endif
#ifndef SOP_KE_LEAF
#define SOP_KE_LEAF 2
#endif
// the same groups when no occurrence of the plan has a third sibling (two
// sibling rows per occurrence instead of three, so more fit in registers)
#ifndef SOP_KE2
#define SOP_KE2 4
#endif
#ifndef SOP_KE_LEAF2
#define SOP_KE_LEAF2 3
#endif
// variables whose Gibbs weights the scan loads together (complex64; 1 holds
// fewer registers and measured faster than 2 or 3)
#ifndef SCAN_PF
#define SCAN_PF 1
#endif
// complex64 waves per SIMD the streaming sampler's register budget is bounded
// for (three-sibling instance, two-sibling instance)
#ifndef STREAM_WAVES_PER_EU
#define STREAM_WAVES_PER_EU 7
#endif
#ifndef STREAM_WAVES_PER_EU2
#define STREAM_WAVES_PER_EU2 8
#endif

// Rows of the region: super-node values [0, S), adjoints [S, 2S), indicator
// derivatives d root / d lambda_{v=u} [2S, 2S + n_ind).  SIB3 = false: no
// occurrence of the plan has a third sibling, so the occurrence walks hold
// two sibling rows each and take larger groups.
template <typename T, bool SIB3>
struct StreamTile {
    DevGraph g;
    RowBuf<T> rb;
    uint32_t adj0, d0;       // first row of the adjoints and of the indicator derivatives
    const uint64_t *ev;      // [W][64] (LDS)
    const cplx<T> *ang;      // [S_ang][64] (LDS)
    const cplx<T> *wfix;     // [S] (LDS copy of the fixed weights)
    int lane;

    // value row of a node reference, zero for a leaf (decoded later by
    // pick): the reference is wave-uniform, so the test is a scalar branch
    // and a batch still issues all of its row loads before the first wait
    __device__ __forceinline__ cplx<T> row(uint32_t r) const {
        if (r != IDENT_REF && (r >> 30) == TAG_NODE) return rb.ld(r & REF_MASK);
        return cplx<T>{T(0), T(0)};
    }
    __device__ __forceinline__ cplx<T> pick(uint32_t r, const cplx<T> &rowval) const {
        return (r >> 30) == TAG_NODE ? rowval : value(r);
    }

    __device__ __forceinline__ cplx<T> value(uint32_t r) const {
        const uint32_t tag = r >> 30, x = r & REF_MASK;
        if (tag == TAG_NODE) return rb.ld(x);
        if (tag == TAG_IND) {
            const uint32_t u = (r >> 26) & 15u, width = ((r >> 24) & 3u) + 1u;
            const uint32_t word = (r >> 6) & 0x3ffffu, shift = r & 63u;
            const bool hit = ((ev[word * WAVE + lane] >> shift) & ((1ull << width) - 1ull)) == static_cast<uint64_t>(u);
            return {hit ? T(1) : T(0), T(0)};
        }
        if (tag == TAG_SLOT) return x < static_cast<uint32_t>(g.S_ang) ? ang[x * WAVE + lane] : wfix[x];
        const uint32_t *rec = g.sel + static_cast<size_t>(x) * SEL_REC;
        const uint32_t fld = cld(rec);
        const uint32_t word = fld >> 8, shift = (fld >> 2) & 63u, width = (fld & 3u) + 1u;
        const uint32_t k = static_cast<uint32_t>((ev[word * WAVE + lane] >> shift) & ((1ull << width) - 1ull));
        const uint32_t s0 = cld(rec + 1), s1 = cld(rec + 2), s2 = cld(rec + 3), s3 = cld(rec + 4);
        const uint32_t sl = k == 0 ? s0 : k == 1 ? s1 : k == 2 ? s2 : k == 3 ? s3 : NO_SLOT;
        return sl == NO_SLOT ? cplx<T>{T(0), T(0)} : wfix[sl];
    }

    // Upward pass on the sum-of-products plan.  A wave takes KB consecutive
    // super-nodes of a level at a time and walks their factors (contiguous in
    // frec) in groups of KF whose rows are all loaded before the first is
    // used; a term's product is formed in registers in factor order, the
    // terms are added in order and a super-node's row is stored once its
    // last factor is in.
    __device__ void forward(const SopPlan &sp, int wave, int nwaves) {
        constexpr int KB = SOP_KB;
        constexpr int KF = sizeof(T) == 4 ? SOP_KF : SOP_KF / 2;
        for (int l = 0; l < sp.L; ++l) {
            const uint32_t n0 = cld(sp.level_ptr + l), n1 = cld(sp.level_ptr + l + 1);
            for (uint32_t b0 = n0 + static_cast<uint32_t>(wave) * KB; b0 < n1; b0 += static_cast<uint32_t>(nwaves) * KB) {
                const uint32_t b1 = b0 + KB < n1 ? b0 + KB : n1;
                const uint32_t f_end = cld(sp.fptr + b1);
                uint32_t t = b0, t_next = cld(sp.fptr + b0 + 1);
                cplx<T> sum{T(0), T(0)}, term{T(1), T(0)};
                for (uint32_t f = cld(sp.fptr + b0); f < f_end; f += KF) {
                    uint64_t rec[KF];
                    cplx<T> v[KF];
#pragma unroll
                    for (int j = 0; j < KF; ++j) rec[j] = f + j < f_end ? cld(sp.frec + f + j) : static_cast<uint64_t>(IDENT_REF);
#pragma unroll
                    for (int j = 0; j < KF; ++j) v[j] = row(static_cast<uint32_t>(rec[j]));
#pragma unroll
                    for (int j = 0; j < KF; ++j) {
                        const uint32_t ff = f + static_cast<uint32_t>(j);
                        if (ff >= f_end) break;
                        while (ff >= t_next) {               // super-node t has all its terms
                            rb.st(t, sum);
                            sum = {T(0), T(0)};
                            ++t;
                            t_next = cld(sp.fptr + t + 1);
                        }
                        term = cmul(term, pick(static_cast<uint32_t>(rec[j]), v[j]));
                        if (rec[j] & SOP_LAST_OF_TERM) {
                            sum = cadd(sum, term);
                            term = {T(1), T(0)};
                        }
                    }
                }
                rb.st(t, sum);                                // every super-node has a factor: t = b1 - 1
            }
            level_sync(nwaves);
        }
    }

    // term of one occurrence: adj[parent] times its (up to three) siblings
    __device__ __forceinline__ cplx<T> occ_term(const uint32_t (&r)[4], const cplx<T> &ap, const cplx<T> &s0,
                                                const cplx<T> &s1, const cplx<T> &s2) const {
        cplx<T> term = ap;
        if (r[1] != NO_SIBLING) term = cmul(term, pick(r[1], s0));
        if (r[2] != NO_SIBLING) term = cmul(term, pick(r[2], s1));
        if (r[3] != NO_SIBLING) term = cmul(term, pick(r[3], s2));
        return term;
    }

    // occurrence record o (parent, siblings); without SIB3 the third sibling
    // is known to be absent and is not read
    __device__ __forceinline__ void load_occ(const SopPlan &sp, uint32_t o, bool in, uint32_t (&r)[4]) const {
        if (in) {
            const uint32_t *q = sp.occ + 4 * static_cast<size_t>(o);
            r[0] = cld(q);
            r[1] = cld(q + 1);
            r[2] = cld(q + 2);
            r[3] = SIB3 ? cld(q + 3) : NO_SIBLING;
        } else {
            r[0] = 0u;
            r[1] = r[2] = r[3] = NO_SIBLING;
        }
    }

    // Adjoint sums of the targets [t0, t1) (super-nodes, then indicator and
    // selector leaves): out(t, sum over the occurrences of t of adj[parent] *
    // siblings), the occurrences in increasing parent order.  The occurrences
    // of the whole range are walked in groups of KE whose row loads (adjoint
    // and sibling rows) are all issued before any term is added.  Without
    // SIB3 no occurrence has a third sibling.
    template <int KE, typename Out>
    __device__ __forceinline__ void pull_group(const SopPlan &sp, uint32_t t0, uint32_t t1, Out out) const {
        const uint32_t e_end = cld(sp.ostart + t1);
        uint32_t t = t0;
        uint32_t t_next = cld(sp.ostart + t0 + 1);      // first occurrence past target t
        double ar = 0.0, ai = 0.0;
        for (uint32_t e = cld(sp.ostart + t0); e < e_end; e += KE) {
            uint32_t rr[KE][4];
            cplx<T> ap[KE], s0[KE], s1[KE], s2[KE];
#pragma unroll
            for (int j = 0; j < KE; ++j) load_occ(sp, e + j, e + j < e_end, rr[j]);
#pragma unroll
            for (int j = 0; j < KE; ++j) {
                ap[j] = rb.ld(adj0 + rr[j][0]);
                s0[j] = row(rr[j][1]);
                s1[j] = row(rr[j][2]);
                s2[j] = SIB3 ? row(rr[j][3]) : cplx<T>{T(0), T(0)};
            }
#pragma unroll
            for (int j = 0; j < KE; ++j) {
                const uint32_t ee = e + static_cast<uint32_t>(j);
                if (ee >= e_end) break;
                while (ee >= t_next) {            // every occurrence of target t is in
                    out(t, cplx<T>{static_cast<T>(ar), static_cast<T>(ai)});
                    ar = 0.0;
                    ai = 0.0;
                    ++t;
                    t_next = cld(sp.ostart + t + 1);
                }
                const cplx<T> term = occ_term(rr[j], ap[j], s0[j], s1[j], s2[j]);
                ar += static_cast<double>(term.re);
                ai += static_cast<double>(term.im);
            }
        }
        for (; t < t1; ++t) {                      // the last target with occurrences, and any without
            out(t, cplx<T>{static_cast<T>(ar), static_cast<T>(ai)});
            ar = 0.0;
            ai = 0.0;
        }
    }
    template <typename Out>
    __device__ __forceinline__ void pull_targets(const SopPlan &sp, uint32_t t0, uint32_t t1, Out out) const {
        constexpr int KE = SIB3 ? SOP_KE : SOP_KE2;
        pull_group<sizeof(T) == 4 ? KE : KE / 2>(sp, t0, t1, out);
    }

    __device__ void backward(const SopPlan &sp, int wave, int nwaves) {
        constexpr int KB = SOP_KB;
        const uint32_t root = static_cast<uint32_t>(sp.root);
        for (int l = sp.L - 1; l >= 0; --l) {
            const uint32_t n0 = cld(sp.level_ptr + l), n1 = cld(sp.level_ptr + l + 1);
            for (uint32_t b0 = n0 + static_cast<uint32_t>(wave) * KB; b0 < n1; b0 += static_cast<uint32_t>(nwaves) * KB) {
                const uint32_t b1 = b0 + KB < n1 ? b0 + KB : n1;
                pull_targets(sp, b0, b1, [&](uint32_t i, cplx<T> v) {
                    rb.st(adj0 + i, i == root ? cplx<T>{T(1), T(0)} : v);
                });
            }
            level_sync(nwaves);
        }
    }

    // acc[u] += sum over the selector occurrences [e, e1) of adj[parent] *
    // siblings * W[slot of value u], in occurrence order; groups of KE
    // occurrences issue their row loads together.  Without SIB3 no occurrence
    // has a third sibling.
    template <int KE>
    __device__ __forceinline__ void sel_occurrences(const SopPlan &sp, uint32_t e, uint32_t e1, uint32_t sel_e0,
                                                    cplx<T> (&acc)[SEL_DOM]) const {
        for (; e < e1; e += KE) {
            uint32_t rr[KE][4];
            uint32_t qe[KE];
            cplx<T> ap[KE], sa[KE], sb[KE], sc[KE];
#pragma unroll
            for (int j = 0; j < KE; ++j) {
                const bool in = e + j < e1;
                load_occ(sp, e + j, in, rr[j]);
                qe[j] = in ? cld(sp.osel + e + j - sel_e0) : 0u;
            }
#pragma unroll
            for (int j = 0; j < KE; ++j) {
                ap[j] = e + j < e1 ? rb.ld(adj0 + rr[j][0]) : cplx<T>{T(0), T(0)};
                sa[j] = row(rr[j][1]);
                sb[j] = row(rr[j][2]);
                sc[j] = SIB3 ? row(rr[j][3]) : cplx<T>{T(0), T(0)};
            }
#pragma unroll
            for (int j = 0; j < KE; ++j) {
                if (e + j >= e1) break;
                const cplx<T> term = occ_term(rr[j], ap[j], sa[j], sb[j], sc[j]);
                const uint32_t *rec = g.sel + static_cast<size_t>(qe[j]) * SEL_REC;
#pragma unroll
                for (int u = 0; u < SEL_DOM; ++u) {
                    const uint32_t sl = cld(rec + 1 + u);
                    if (sl != NO_SLOT) acc[u] = cadd(acc[u], cmul(term, wfix[sl]));
                }
            }
        }
    }

    // d root / d lambda_{v=u}, one wave per variable: the adjoint sums of v's
    // indicator leaves into its D rows, then every occurrence of v's selector
    // leaves (contiguous in the plan, in groups of KE whose row loads issue
    // together) adds its term times the occurrence's selector weight for each
    // value u.  Only D rows are stored; no barrier inside.  With `decide`,
    // each variable's values d[0..dom) (at most SEL_DOM, as stored) are then
    // handed to dec(v, d, dom) while still in registers.
    template <typename Decide>
    __device__ void leaf_derivatives(const SopPlan &sp, int wave, int nwaves, bool decide, Decide &&dec) {
        constexpr int KL = SIB3 ? SOP_KE_LEAF : SOP_KE_LEAF2;
        constexpr int KE = sizeof(T) == 4 ? KL : KL / 2 > 0 ? KL / 2 : 1;
        const uint32_t M = static_cast<uint32_t>(sp.S);
        const uint32_t s0t = M + static_cast<uint32_t>(g.n_ind);   // first selector target
        const uint32_t sel_e0 = cld(sp.ostart + s0t);               // first selector occurrence
        for (int v = wave; v < g.n_vars; v += nwaves) {
            const uint32_t base = cld(g.ind_base + v), dom = cld(g.ind_base + v + 1) - base;
            const uint32_t q0 = cld(g.vsel_ptr + v), q1 = cld(g.vsel_ptr + v + 1);
            // indicator leaves: walked unless v has none with an occurrence and
            // all of its values are covered by the selector accumulators
            const bool ind_occ = cld(sp.ostart + M + base) != cld(sp.ostart + M + base + dom);
            const bool walk_ind = dom > 0 && (ind_occ || q0 == q1 || dom > static_cast<uint32_t>(SEL_DOM));
            cplx<T> acc[SEL_DOM];
#pragma unroll
            for (int u = 0; u < SEL_DOM; ++u) acc[u] = {T(0), T(0)};
            if (walk_ind)
                pull_targets(sp, M + base, M + base + dom, [&](uint32_t i, cplx<T> val) {
                    rb.st(d0 + (i - M), val);
                    const uint32_t u = i - M - base;
#pragma unroll
                    for (int k = 0; k < SEL_DOM; ++k)
                        if (u == static_cast<uint32_t>(k)) acc[k] = val;
                });
            if (q0 != q1) {
                const uint32_t e0 = cld(sp.ostart + s0t + q0), e1 = cld(sp.ostart + s0t + q1);
                sel_occurrences<KE>(sp, e0, e1, sel_e0, acc);
#pragma unroll
                for (int u = 0; u < SEL_DOM; ++u)
                    if (static_cast<uint32_t>(u) < dom) rb.st(d0 + base + u, acc[u]);
            }
            if (decide) dec(v, acc, static_cast<int>(dom));
        }
    }
};

// complex64: the kernel waits on dependent row loads and more resident waves
// hide more of it, against more spills (1,024,000 8-qubit samples on the
// sum-of-products plan with three sibling rows per occurrence: 4 waves 546
// ms, 5 waves 509 ms, 6 waves 484 ms; with two, 6 and 7 waves both 461 ms,
// and with the scan loading one variable's weights at a time, 8 waves (64
// VGPRs) 453 ms against 456 ms at 6).  The three-sibling instance runs 7
// waves (72 VGPRs): 1,000,192 32-qubit samples 1980 / 1872 / 1870 ms at
// 6 / 7 / 8 waves, but 8 slows the 32-qubit p=2 batch (2715 / 2758 / 2866 ms).
// SIB3 = false when the plan has no occurrence with a third sibling: the
// downward pass then holds two sibling rows per occurrence in its groups of
// 4 and the leaf step takes groups of 3 instead of 2 (groups of 5 and 4
// measured slower); the chains are the same.
template <typename T, bool SIB3>
__global__ __launch_bounds__(MAX_BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (SIB3 ? STREAM_WAVES_PER_EU : STREAM_WAVES_PER_EU2) : 1, 8))) void k_sample_stream(DevGraph g, SopPlan sp, const double *theta,
                                                         const Weight<T> *wfix, cplx<T> *vals, size_t per_wg,
                                                         SampleArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *ev_s = reinterpret_cast<uint64_t *>(smem);
    cplx<T> *ang_s = reinterpret_cast<cplx<T> *>(smem + static_cast<size_t>(g.W) * WAVE * 8);
    cplx<T> *fix_s = ang_s + static_cast<size_t>(g.S_ang) * WAVE;
    uint64_t *mask_s = reinterpret_cast<uint64_t *>(fix_s + g.S);   // [mask_words][64] change bits
    __shared__ int64_t s_chain[WAVE];
    __shared__ int32_t s_pos[WAVE];
    __shared__ uint32_t s_sweep[WAVE];
    __shared__ int32_t s_emitted[WAVE];
    __shared__ int64_t s_rounds[WAVE];

    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = static_cast<int>(uniform_u32(threadIdx.x / WAVE));
    const int nwaves = blockDim.x / WAVE;
    const bool decide_all = sp.mask_words > 0 && !a.seq_scan;
    cplx<T> *val = vals + per_wg * blockIdx.x;
    cplx<T> *D = val + 2 * static_cast<size_t>(sp.S) * WAVE;    // [n_ind][64]
    for (int s2 = threadIdx.x; s2 < g.S; s2 += blockDim.x) fix_s[s2] = wval(wfix[s2]);
    const uint32_t N = static_cast<uint32_t>(sp.S);
    StreamTile<T, SIB3> t{g, RowBuf<T>(val, per_wg / WAVE, lane), N, 2 * N, ev_s, ang_s, fix_s, lane};
    const int64_t stride = static_cast<int64_t>(gridDim.x) * WAVE;
    const uint32_t total_sweeps = static_cast<uint32_t>(a.burn_in) +
                                  static_cast<uint32_t>(a.spc) * static_cast<uint32_t>(a.thin);
    const uint64_t xmask = g.n_qubits >= 64 ? ~0ull : ((1ull << g.n_qubits) - 1ull);

    auto init_chain = [&](int64_t ch) {      // wave 0
        s_chain[lane] = ch;
        s_pos[lane] = a.first_var;
        s_sweep[lane] = 0;
        s_emitted[lane] = 0;
        s_rounds[lane] = 0;
        for (int w = 0; w < g.W; ++w)
            ev_s[w * WAVE + lane] = (ch >= 0 && a.init_states) ? a.init_states[ch * g.W + w] : 0ull;
        if (ch >= 0 && !a.init_states) {
            uint64_t x = 0;
            for (int q = 0; q < g.n_qubits; ++q)
                if (rng_uniform(a.seed, a.chain_offset + static_cast<uint64_t>(ch), INIT_SWEEP, static_cast<uint64_t>(q)) < 0.5)
                    x |= (1ull << q);
            ev_s[lane] = x;
        }
    };

    if (wave == 0) {
        const int64_t ch = static_cast<int64_t>(blockIdx.x) * WAVE + lane;
        init_chain(ch < a.total_chains ? ch : -1);
    }
    __syncthreads();

    for (;;) {
        const int64_t ch = s_chain[lane];
        if (!__syncthreads_or(ch >= 0 ? 1 : 0)) break;
        const int p = ch >= 0 ? static_cast<int>(ch / a.cpp) : 0;
        const double *trow = theta + static_cast<int64_t>(p) * g.K;
        for (int s2 = wave; s2 < g.S_ang; s2 += nwaves) {
            double re, im;
            slot_value(g.slots[s2], trow, nullptr, re, im);
            ang_s[s2 * WAVE + lane] = {static_cast<T>(re), static_cast<T>(im)};
        }
        if (decide_all)
            for (int w2 = wave; w2 < sp.mask_words; w2 += nwaves) mask_s[w2 * WAVE + lane] = 0ull;
        __syncthreads();
        t.forward(sp, wave, nwaves);
        t.backward(sp, wave, nwaves);
        // Decisions: the Gibbs choice of every variable at its first visit in
        // this round (variables before the chain's position come after the
        // sweep boundary), taken in the leaf step by the wave that has the
        // variable's derivatives in registers -- they stay valid up to the
        // first change; a changed value sets the variable's bit in the
        // chain's change mask, and the scan jumps to the first set bit
        // instead of visiting the variables one by one.
        const int32_t pos0 = s_pos[lane];
        const uint32_t sw0 = s_sweep[lane];
        t.leaf_derivatives(sp, wave, nwaves, decide_all, [&](int v, const cplx<T> (&d)[SEL_DOM], int dom) {
            if (ch < 0 || v < a.first_var) return;
            const uint32_t fld = cld(g.var_field + v);
            const uint32_t word = fld >> 8, shift = (fld >> 2) & 63u, width = (fld & 3u) + 1u;
            const uint32_t cur = static_cast<uint32_t>((ev_s[word * WAVE + lane] >> shift) & ((1ull << width) - 1ull));
            double w[SEL_DOM];
#pragma unroll
            for (int u = 0; u < SEL_DOM; ++u) w[u] = u < dom ? gibbs_weight(d[u]) : 0.0;
            const uint32_t sw = sw0 + (v < pos0 ? 1u : 0u);
            const double r = rng_uniform(a.seed, a.chain_offset + static_cast<uint64_t>(ch), a.first_sweep + sw, static_cast<uint64_t>(v));
            if (gibbs_choice(w, dom, cur, r) != cur)
                atomicOr(reinterpret_cast<unsigned long long *>(mask_s + (v >> 6) * WAVE + lane), 1ull << (v & 63));
        });
        __syncthreads();

        if (wave == 0 && ch >= 0) {
            s_rounds[lane] += 1;
            int32_t pos = s_pos[lane];
            uint32_t sweep = s_sweep[lane];
            int32_t emitted = s_emitted[lane];
            bool done = false;
            // the state after a completed sweep: a sample when past the
            // burn-in and on the thinning stride
            auto end_sweep = [&]() -> bool {
                pos = a.first_var;
                sweep += 1;
                if (sweep > static_cast<uint32_t>(a.burn_in) &&
                    (sweep - static_cast<uint32_t>(a.burn_in)) % static_cast<uint32_t>(a.thin) == 0u) {
                    const int64_t S = static_cast<int64_t>(a.cpp) * a.spc;
                    const int64_t idx = static_cast<int64_t>(p) * S + (ch % a.cpp) * a.spc + emitted;
                    const uint64_t x = ev_s[lane] & xmask;
                    a.samples[idx * a.nwq] = x;
                    for (int w2 = 1; w2 < a.nwq; ++w2) a.samples[idx * a.nwq + w2] = 0ull;
                    if (a.states_out)
                        for (int w2 = 0; w2 < g.W; ++w2) a.states_out[idx * g.W + w2] = ev_s[w2 * WAVE + lane];
                    if (a.cost_out) {
                        a.cost_out[idx] = maxcut_cost(a, x, g.n_qubits);
                    }
                    emitted += 1;
                }
                return sweep >= total_sweeps;
            };
            bool scan = true;
            if (decide_all) {
                // first changed variable in [lo, hi), or -1
                auto first_set = [&](int lo, int hi) -> int {
                    for (int v = lo; v < hi;) {
                        const int off = v & 63;
                        uint64_t m = mask_s[(v >> 6) * WAVE + lane] >> off;
                        const int lim = hi - v < 64 - off ? hi - v : 64 - off;
                        if (lim < 64) m &= (1ull << lim) - 1ull;
                        if (m) return v + __builtin_ctzll(m);
                        v += 64 - off;
                    }
                    return -1;
                };
                // the recorded change at v, decided again from its derivatives
                auto apply = [&](int v) {
                    const uint32_t bk = g.ind_base[v];
                    const int dom = static_cast<int>(g.ind_base[v + 1] - bk);
                    double w[SEL_DOM];
#pragma unroll
                    for (int u = 0; u < SEL_DOM; ++u)
                        w[u] = u < dom ? gibbs_weight(D[static_cast<size_t>(bk + u) * WAVE + lane]) : 0.0;
                    const uint32_t fld = g.var_field[v];
                    const uint32_t word = fld >> 8, shift = (fld >> 2) & 63u, width = (fld & 3u) + 1u;
                    const uint64_t fmask = (1ull << width) - 1ull;
                    const uint64_t wv = ev_s[word * WAVE + lane];
                    const uint32_t cur = static_cast<uint32_t>((wv >> shift) & fmask);
                    const double r = rng_uniform(a.seed, a.chain_offset + static_cast<uint64_t>(ch), a.first_sweep + sweep, static_cast<uint64_t>(v));
                    const uint32_t pick = gibbs_choice(w, dom, cur, r);
                    ev_s[word * WAVE + lane] = (wv & ~(fmask << shift)) | (static_cast<uint64_t>(pick) << shift);
                };
                const int pos0 = pos;
                const int vs = first_set(pos0, g.n_vars);
                if (vs >= 0) {                       // a change later in this sweep
                    apply(vs);
                    pos = vs + 1;
                    if (pos == g.n_vars) done = end_sweep();
                    scan = false;
                } else {
                    done = end_sweep();              // the rest of the sweep keeps every value
                    if (done) {
                        scan = false;
                    } else {
                        const int vb = first_set(a.first_var, pos0);
                        if (vb >= 0) {               // a change in the next sweep, before pos0
                            apply(vb);
                            pos = vb + 1;
                            scan = false;
                        } else {
                            pos = pos0;              // a whole cycle unchanged: scan on from pos0
                        }
                    }
                }
            }
            // Gibbs weights of the next PF variables, loaded together (the
            // derivatives do not change until the state does)
            constexpr int PF = sizeof(T) == 4 ? SCAN_PF : 2;
            double wpf[PF][SEL_DOM];
            int pf_pos = -1;
            for (; scan && !done;) {
                const int v = pos;
                if (pf_pos < 0 || v < pf_pos || v >= pf_pos + PF) {
                    pf_pos = v;
                    cplx<T> dv[PF][SEL_DOM];
#pragma unroll
                    for (int k = 0; k < PF; ++k) {
                        const int vk = v + k < g.n_vars ? v + k : v;
                        const uint32_t bk = g.ind_base[vk], dk = g.ind_base[vk + 1] - bk;
#pragma unroll
                        for (int u = 0; u < SEL_DOM; ++u)
                            dv[k][u] = D[static_cast<size_t>(bk + (static_cast<uint32_t>(u) < dk ? u : 0)) * WAVE + lane];
                    }
#pragma unroll
                    for (int k = 0; k < PF; ++k)
#pragma unroll
                        for (int u = 0; u < SEL_DOM; ++u) {
                            const double re = static_cast<double>(dv[k][u].re), im = static_cast<double>(dv[k][u].im);
                            wpf[k][u] = __dadd_rn(__dmul_rn(re, re), __dmul_rn(im, im));
                        }
                }
                const uint32_t fld = g.var_field[v];
                const uint32_t word = fld >> 8, shift = (fld >> 2) & 63u, width = (fld & 3u) + 1u;
                const uint64_t fmask = (1ull << width) - 1ull;
                const uint32_t cur = static_cast<uint32_t>((ev_s[word * WAVE + lane] >> shift) & fmask);
                const uint32_t base = g.ind_base[v];
                const int dom = static_cast<int>(g.ind_base[v + 1] - base);
                const int kk = v - pf_pos;
                auto weight = [&](int u) -> double {
                    if (u < SEL_DOM) {
                        double w = 0.0;
#pragma unroll
                        for (int k = 0; k < PF; ++k)
#pragma unroll
                            for (int u2 = 0; u2 < SEL_DOM; ++u2)
                                if (k == kk && u2 == u) w = wpf[k][u2];
                        return w;
                    }
                    const cplx<T> d = D[static_cast<size_t>(base + u) * WAVE + lane];
                    const double re = static_cast<double>(d.re), im = static_cast<double>(d.im);
                    return __dadd_rn(__dmul_rn(re, re), __dmul_rn(im, im));
                };
                double total = 0.0;
                for (int u = 0; u < dom; ++u) total = __dadd_rn(total, weight(u));
                uint32_t pick = cur;
                if (total > 0.0) {
                    const double r = rng_uniform(a.seed, a.chain_offset + static_cast<uint64_t>(ch), a.first_sweep + sweep, static_cast<uint64_t>(v));
                    const double target = __dmul_rn(r, total);
                    double acc = 0.0;
                    int last_pos = -1, chosen = -1;
                    for (int u = 0; u < dom; ++u) {
                        const double w = weight(u);
                        acc = __dadd_rn(acc, w);
                        if (w > 0.0) last_pos = u;
                        if (target < acc) {
                            chosen = u;
                            break;
                        }
                    }
                    if (chosen < 0) chosen = last_pos;
                    if (chosen >= 0) pick = static_cast<uint32_t>(chosen);
                }
                const bool changed = pick != cur;
                if (changed) {
                    uint64_t wv = ev_s[word * WAVE + lane];
                    ev_s[word * WAVE + lane] = (wv & ~(fmask << shift)) | (static_cast<uint64_t>(pick) << shift);
                }
                pos += 1;
                if (pos == g.n_vars && end_sweep()) {
                    done = true;
                    break;
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
// Gibbs sampler, LDS-resident node-parallel variant
// ---------------------------------------------------------------------------
//
// One wavefront works on CPW chains at once; each chain owns 64/CPW lanes and
// a private LDS block holding every node value and adjoint of the DAG plan,
// the indicator derivatives, its weights, its evidence words and its
// bookkeeping.  Lanes split the nodes of a level, so nothing but the DAG
// structure (read-only, cached) and the outputs touches global memory.

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~static_cast<size_t>(15); }

template <typename T>
__host__ __device__ inline size_t chain_values(int N, int n_ind, int S, int n_sel, int max_edges) {
    return 2 * static_cast<size_t>(N) + n_ind + S + n_sel + max_edges;
}

template <typename T>
__host__ __device__ inline size_t chain_lds_bytes(int N, int n_ind, int S, int n_sel, int max_edges, int W) {
    return al16(al16(chain_values<T>(N, n_ind, S, n_sel, max_edges) * sizeof(cplx<T>)) + static_cast<size_t>(W) * 8 +
                8 * 8);
}

// per-workgroup level table in LDS: level_ptr[L+1], level_prod[L+1], first edge[L+1]
__host__ __device__ inline size_t level_meta_bytes(int L) { return al16(3 * (static_cast<size_t>(L) + 1) * 4); }

template <typename T>
struct ChainView {
    cplx<T> *val, *adj, *D, *sv, *selv, *tmp;
    uint64_t *ev;
    int64_t *st;      // 0 chain (-1: none), 1 pos, 2 sweep, 3 emitted, 4 rounds, 5 param set, 6 restage

    __device__ __forceinline__ bool ind_hit(uint32_t r) const {
        const uint32_t u = (r >> 26) & 15u, width = ((r >> 24) & 3u) + 1u;
        const uint32_t word = (r >> 6) & 0x3ffffu, shift = r & 63u;
        return ((ev[word] >> shift) & ((1ull << width) - 1ull)) == static_cast<uint64_t>(u);
    }
    __device__ __forceinline__ cplx<T> value(uint32_t r) const {
        const uint32_t tag = r >> 30;
        if (tag == TAG_NODE) return val[r & REF_MASK];
        if (tag == TAG_IND) return {ind_hit(r) ? T(1) : T(0), T(0)};
        if (tag == TAG_SEL) return selv[r & REF_MASK];
        return sv[r & REF_MASK];
    }
    // unified reference (index into [node | slot | selector] values, or an
    // indicator): both loads are issued unconditionally and the result is
    // selected, so lanes holding different kinds of children do not serialise
    __device__ __forceinline__ cplx<T> uval(uint32_t r) const {
        const uint32_t tag = r >> 30;
        const cplx<T> v = val[tag == TAG_NODE ? r : 0u];
        const uint32_t word = tag == TAG_IND ? ((r >> 6) & 0x3ffffu) : 0u;
        const uint64_t w = ev[word];
        const uint32_t u = (r >> 26) & 15u, width = ((r >> 24) & 3u) + 1u, shift = r & 63u;
        const bool hit = ((w >> shift) & ((1ull << width) - 1ull)) == static_cast<uint64_t>(u);
        if (tag == TAG_IND) return {hit ? T(1) : T(0), T(0)};
        return v;
    }
};

// Output of one emitted sample (the state words are read from `ev`, except
// that word `cw` is replaced by `cval` when cw < W).
__device__ inline void emit_sample(const DevGraph &g, const SampleArgs &a, int64_t idx, const uint64_t *ev,
                                   int cw, uint64_t cval, uint64_t xmask) {
    const uint64_t w0 = cw == 0 ? cval : ev[0];
    const uint64_t x = w0 & xmask;
    a.samples[idx * a.nwq] = x;
    for (int w2 = 1; w2 < a.nwq; ++w2) a.samples[idx * a.nwq + w2] = 0ull;
    if (a.states_out)
        for (int w2 = 0; w2 < g.W; ++w2) a.states_out[idx * g.W + w2] = w2 == cw ? cval : ev[w2];
    if (a.cost_out) {
        a.cost_out[idx] = maxcut_cost(a, x, g.n_qubits);
    }
}

// The LDS-resident kernels run one wavefront per workgroup: the LDS accesses
// of a wave execute in order, so lanes only need the compiler to keep program
// order here.  A wavefront-scope fence does that without waiting for
// outstanding global loads (a workgroup barrier would also wait for the
// records prefetched for later levels).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// the lanes working on one chain meet: one wavefront, or the workgroup
template <int WPC>
__device__ __forceinline__ void chain_sync() {
    if constexpr (WPC == 1) wave_sync();
    else __syncthreads();
}

template <typename T, int CPW, int WPC>
__global__ __launch_bounds__(WAVE * WPC) void k_sample_lds(DevGraph g, LdsPlan lp, const double *theta,
                                                     const double *noise, SampleArgs a, uint32_t chain_bytes) {
    extern __shared__ __align__(16) unsigned char smem[];
    static_assert(WPC == 1 || CPW == 1, "several waves work on one chain, or one wave on several");
    constexpr int LPC = WAVE * WPC / CPW;     // lanes per chain in the node passes
    constexpr int DPC = WAVE / CPW;           // lanes per chain in the Gibbs decisions (wave 0 only)
    const int lane = threadIdx.x;
    const int sub = lane / LPC;
    const int cl = lane - sub * LPC;
    const int wl = lane & (WAVE - 1);
    const int dsub = wl / DPC;
    const int dcl = wl - dsub * DPC;
    const int L = lp.L;
    uint32_t *lv_ptr = reinterpret_cast<uint32_t *>(smem);
    uint32_t *lv_prod = lv_ptr + (L + 1);
    uint32_t *lv_edge = lv_prod + (L + 1);
    for (int l = lane; l <= L; l += WAVE * WPC) {
        lv_ptr[l] = lp.level_ptr[l];
        lv_prod[l] = l < L ? lp.level_prod[l] : lp.level_ptr[L];
        lv_edge[l] = lp.estart[lp.level_ptr[l]];
    }
    unsigned char *blk = smem + level_meta_bytes(L) + static_cast<size_t>(sub) * chain_bytes;
    ChainView<T> c;
    c.val = reinterpret_cast<cplx<T> *>(blk);      // [node | slot | selector] values
    c.sv = c.val + lp.N;
    c.selv = c.sv + g.S;
    c.adj = c.selv + g.n_sel;
    c.D = c.adj + lp.N;
    c.tmp = c.D + g.n_ind;
    c.ev = reinterpret_cast<uint64_t *>(
        blk + al16(chain_values<T>(lp.N, g.n_ind, g.S, g.n_sel, lp.max_edges) * sizeof(cplx<T>)));
    c.st = reinterpret_cast<int64_t *>(c.ev + g.W);
    const double *nz = noise ? noise : g.noise_default;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * CPW;
    const uint32_t total_sweeps = static_cast<uint32_t>(a.burn_in) +
                                  static_cast<uint32_t>(a.spc) * static_cast<uint32_t>(a.thin);
    const uint64_t xmask = g.n_qubits >= 64 ? ~0ull : ((1ull << g.n_qubits) - 1ull);
    const int shift_sub = dsub * DPC;
    const uint64_t gmask = DPC == WAVE ? ~0ull : (((1ull << DPC) - 1ull) << shift_sub);
    const uint32_t T_all = static_cast<uint32_t>(lp.N + g.n_ind + g.n_sel);
    const uint32_t leaf_e0 = lp.estart[lp.N], leaf_e1 = lp.estart[T_all];

    auto init_chain = [&](int64_t ch) {      // lane cl == 0 of the chain group
        c.st[0] = ch;
        c.st[1] = 0;
        c.st[2] = 0;
        c.st[3] = 0;
        c.st[4] = 0;
        c.st[5] = ch >= 0 ? ch / a.cpp : 0;
        c.st[6] = 1;
        for (int w = 0; w < g.W; ++w) c.ev[w] = (ch >= 0 && a.init_states) ? a.init_states[ch * g.W + w] : 0ull;
        if (ch >= 0 && !a.init_states) {
            uint64_t x = 0;
            for (int q = 0; q < g.n_qubits; ++q)
                if (rng_uniform(a.seed, a.chain_offset + static_cast<uint64_t>(ch), INIT_SWEEP, static_cast<uint64_t>(q)) < 0.5)
                    x |= (1ull << q);
            c.ev[0] = x;
        }
    };
    // adj[parent] * value(sibling) of one parent edge
    auto edge_term = [&](uint64_t rr) {
        const cplx<T> t = c.adj[static_cast<uint32_t>(rr)];
        const uint32_t sib = static_cast<uint32_t>(rr >> 32);
        const cplx<T> sv = c.uval(sib);
        return sib == NO_SIBLING ? t : cmul(t, sv);
    };
    auto sum_tmp = [&](uint32_t s0, uint32_t s1) {
        double ar = 0.0, ai = 0.0;
        for (uint32_t q = s0; q < s1; ++q) {
            ar += static_cast<double>(c.tmp[q].re);
            ai += static_cast<double>(c.tmp[q].im);
        }
        return cplx<T>{static_cast<T>(ar), static_cast<T>(ai)};
    };
    // first record of level l for this lane (prefetch helpers)
    auto fwd_first = [&](int l) -> uint64_t {
        if (l >= L) return ~0ull;
        const uint32_t i = lv_ptr[l] + cl;
        return i < lv_ptr[l + 1] ? lp.fwd_u[i] : ~0ull;
    };
    auto edge_first = [&](int l) -> uint64_t {
        if (l < 0) return 0ull;
        const uint32_t e = lv_edge[l] + cl;
        return e < lv_edge[l + 1] ? lp.edg_u[e] : 0ull;
    };
    auto bound_first = [&](int l) -> uint64_t {
        if (l < 0) return 0ull;
        const uint32_t i = lv_ptr[l] + cl;
        return i < lv_ptr[l + 1] ? (static_cast<uint64_t>(lp.estart[i]) | (static_cast<uint64_t>(lp.estart[i + 1]) << 32))
                                 : 0ull;
    };

    if (cl == 0) {
        const int64_t ch = static_cast<int64_t>(blockIdx.x) * CPW + sub;
        init_chain(ch < a.total_chains ? ch : -1);
    }
    chain_sync<WPC>();

    for (;;) {
        if (c.st[6] != 0) {                  // weights of a chain that just started
            const double *trow = theta + c.st[5] * g.K;
            for (int s = cl; s < g.S; s += LPC) {
                double re, im;
                slot_value(g.slots[s], trow, nz, re, im);
                c.sv[s] = {static_cast<T>(re), static_cast<T>(im)};
            }
        }
        chain_sync<WPC>();
        if (cl == 0) c.st[6] = 0;
        const bool active = c.st[0] >= 0;
        if (__ballot(active) == 0ull) break;

        // ---- selector leaves of this round's state
        if (active) {
            for (int q = cl; q < g.n_sel; q += LPC) {
                const uint4 sr = *reinterpret_cast<const uint4 *>(g.sel + static_cast<size_t>(q) * SEL_REC);
                const uint32_t s4 = g.sel[static_cast<size_t>(q) * SEL_REC + 4];
                const uint32_t word = sr.x >> 8, shift = (sr.x >> 2) & 63u, width = (sr.x & 3u) + 1u;
                const uint32_t k = static_cast<uint32_t>((c.ev[word] >> shift) & ((1ull << width) - 1ull));
                const uint32_t sl = k == 0 ? sr.y : k == 1 ? sr.z : k == 2 ? sr.w : k == 3 ? s4 : NO_SLOT;
                c.selv[q] = sl == NO_SLOT ? cplx<T>{T(0), T(0)} : c.sv[sl];
            }
        }
        chain_sync<WPC>();

        // ---- upward pass; the first record of a level is loaded two levels ahead
        {
            uint64_t r0 = active ? fwd_first(0) : ~0ull;
            uint64_t r1 = active ? fwd_first(1) : ~0ull;
            for (int l = 0; l < L; ++l) {
                const uint64_t r2 = active ? fwd_first(l + 2) : ~0ull;
                const uint32_t n1 = lv_ptr[l + 1], np = lv_prod[l];
                if (active) {
                    uint64_t rec = r0;
                    for (uint32_t i = lv_ptr[l] + cl; i < n1; i += LPC) {
                        const uint32_t inext = i + LPC;
                        const uint64_t rnext = inext < n1 ? lp.fwd_u[inext] : ~0ull;
                        const uint32_t ra = static_cast<uint32_t>(rec), rb = static_cast<uint32_t>(rec >> 32);
                        const cplx<T> va = c.uval(ra);
                        const cplx<T> vb = c.uval(rb);
                        const bool prod = i >= np;
                        const cplx<T> pr = cmul(va, vb), sm = cadd(va, vb);
                        c.val[i] = rb == IDENT_REF ? va : (prod ? pr : sm);
                        rec = rnext;
                    }
                }
                r0 = r1;
                r1 = r2;
                chain_sync<WPC>();
            }
        }
        // ---- downward pass, level by level: every parent edge of the level's
        // nodes in parallel into tmp, then each node sums its edge range
        {
            uint64_t e0r = active ? edge_first(L - 1) : 0ull, e1r = active ? edge_first(L - 2) : 0ull;
            uint64_t b0r = active ? bound_first(L - 1) : 0ull, b1r = active ? bound_first(L - 2) : 0ull;
            for (int l = L - 1; l >= 0; --l) {
                const uint64_t e2r = active ? edge_first(l - 2) : 0ull;
                const uint64_t b2r = active ? bound_first(l - 2) : 0ull;
                const uint32_t eb0 = lv_edge[l], eb1 = lv_edge[l + 1];
                if (active) {
                    uint64_t rr = e0r;
                    for (uint32_t e = eb0 + cl; e < eb1; e += LPC) {
                        const uint32_t enext = e + LPC;
                        const uint64_t rnext = enext < eb1 ? lp.edg_u[enext] : 0ull;
                        c.tmp[e - eb0] = edge_term(rr);
                        rr = rnext;
                    }
                }
                chain_sync<WPC>();
                if (active) {
                    const uint32_t n1 = lv_ptr[l + 1];
                    uint64_t bb = b0r;
                    for (uint32_t i = lv_ptr[l] + cl; i < n1; i += LPC) {
                        const uint32_t inext = i + LPC;
                        const uint64_t bnext =
                            inext < n1 ? (static_cast<uint64_t>(lp.estart[inext]) |
                                          (static_cast<uint64_t>(lp.estart[inext + 1]) << 32))
                                       : 0ull;
                        c.adj[i] = i == static_cast<uint32_t>(lp.root)
                                       ? cplx<T>{T(1), T(0)}
                                       : sum_tmp(static_cast<uint32_t>(bb) - eb0, static_cast<uint32_t>(bb >> 32) - eb0);
                        bb = bnext;
                    }
                }
                e0r = e1r;
                e1r = e2r;
                b0r = b1r;
                b1r = b2r;
                chain_sync<WPC>();
            }
            // leaves: every parent edge of indicator and selector leaves, then
            // d root / d lambda_{v=u} per variable
            if (active) {
                for (uint32_t e = leaf_e0 + cl; e < leaf_e1; e += LPC) c.tmp[e - leaf_e0] = edge_term(lp.edg_u[e]);
            }
            chain_sync<WPC>();
            if (active) {
                for (int t0 = cl; t0 < g.n_ind; t0 += LPC) {
                    double ar = 0.0, ai = 0.0;
                    const uint32_t j1 = lp.dstart[t0 + 1];
                    for (uint32_t j = lp.dstart[t0]; j < j1; ++j) {
                        const uint64_t dt = lp.dterm[j];
                        const uint32_t sl = static_cast<uint32_t>(dt >> 32);
                        const cplx<T> term = c.tmp[static_cast<uint32_t>(dt)];
                        const cplx<T> wv = c.sv[sl == NO_SLOT ? 0u : sl];
                        const cplx<T> x = sl == NO_SLOT ? term : cmul(term, wv);
                        ar += static_cast<double>(x.re);
                        ai += static_cast<double>(x.im);
                    }
                    c.D[t0] = {static_cast<T>(ar), static_cast<T>(ai)};
                }
            }
            chain_sync<WPC>();
        }

        // ---- Gibbs decisions: lane k decides the k-th next variable of the
        // scan; the first lane whose decision changes the state ends the round.
        // With several waves on one chain, wave 0 alone decides.
        if (active && (WPC == 1 || lane < WAVE)) {
            const int64_t ch = c.st[0];
            const int p = static_cast<int>(c.st[5]);
            int64_t pos = c.st[1];
            uint32_t sweep = static_cast<uint32_t>(c.st[2]);
            int32_t emitted = static_cast<int32_t>(c.st[3]);
            const int V = g.n_vars - a.first_var;      // variables the scan visits
            const int64_t S = static_cast<int64_t>(a.cpp) * a.spc;
            const int64_t out0 = static_cast<int64_t>(p) * S + (ch % a.cpp) * a.spc;
            bool done = false;
            for (;;) {
                const int64_t t = pos + dcl;
                const uint32_t sw = sweep + static_cast<uint32_t>(t / V);
                const int v = a.first_var + static_cast<int>(t % V);
                const bool valid = sw < total_sweeps;
                uint32_t cur = 0, pick = 0, word = 0, shift = 0;
                uint64_t fmask = 0;
                if (valid) {
                    const uint32_t fld = g.var_field[v];
                    word = fld >> 8;
                    shift = (fld >> 2) & 63u;
                    fmask = (1ull << ((fld & 3u) + 1u)) - 1ull;
                    cur = static_cast<uint32_t>((c.ev[word] >> shift) & fmask);
                    pick = cur;
                    const uint32_t base = g.ind_base[v];
                    const int dom = static_cast<int>(g.ind_base[v + 1] - base);
                    double total = 0.0;
                    for (int u = 0; u < dom; ++u) {
                        const cplx<T> d = c.D[base + u];
                        const double re = static_cast<double>(d.re), im = static_cast<double>(d.im);
                        total = __dadd_rn(total, __dadd_rn(__dmul_rn(re, re), __dmul_rn(im, im)));
                    }
                    if (total > 0.0) {
                        const double r = rng_uniform(a.seed, a.chain_offset + static_cast<uint64_t>(ch), a.first_sweep + sw, static_cast<uint64_t>(v));
                        const double target = __dmul_rn(r, total);
                        double acc = 0.0;
                        int last_pos = -1, chosen = -1;
                        for (int u = 0; u < dom; ++u) {
                            const cplx<T> d = c.D[base + u];
                            const double re = static_cast<double>(d.re), im = static_cast<double>(d.im);
                            const double w = __dadd_rn(__dmul_rn(re, re), __dmul_rn(im, im));
                            acc = __dadd_rn(acc, w);
                            if (w > 0.0) last_pos = u;
                            if (target < acc) {
                                chosen = u;
                                break;
                            }
                        }
                        if (chosen < 0) chosen = last_pos;
                        if (chosen >= 0) pick = static_cast<uint32_t>(chosen);
                    }
                }
                const bool changed = valid && pick != cur;
                const uint64_t chg = (__ballot(changed) & gmask) >> shift_sub;
                const uint64_t vld = (__ballot(valid) & gmask) >> shift_sub;
                const int f = chg ? __ffsll(static_cast<unsigned long long>(chg)) - 1 : -1;
                const int last = vld ? 63 - __clzll(static_cast<unsigned long long>(vld)) : -1;
                const int end = f >= 0 ? f : last;
                bool emit = false;
                if (valid && dcl <= end && v == g.n_vars - 1) {
                    const uint32_t done_sw = sw + 1;
                    emit = done_sw > static_cast<uint32_t>(a.burn_in) &&
                           (done_sw - static_cast<uint32_t>(a.burn_in)) % static_cast<uint32_t>(a.thin) == 0u;
                }
                const uint64_t em = (__ballot(emit) & gmask) >> shift_sub;
                const uint64_t newword = (dcl == f) ? ((c.ev[word] & ~(fmask << shift)) |
                                                      (static_cast<uint64_t>(pick) << shift)) : 0ull;
                if (emit) {
                    const int rank = __popcll(static_cast<unsigned long long>(em & ((1ull << dcl) - 1ull)));
                    emit_sample(g, a, out0 + emitted + rank, c.ev, dcl == f ? static_cast<int>(word) : g.W,
                                newword, xmask);
                }
                emitted += __popcll(static_cast<unsigned long long>(em));
                // one wavefront per workgroup: LDS accesses of the wave execute in
                // order; the fences keep the compiler from reordering them and wait
                // for completion (every emission reads the old state first)
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
                if (dcl == f) c.ev[word] = newword;
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
                if (end < 0) {                   // nothing left to decide
                    done = true;
                    break;
                }
                const int64_t tn = pos + end + 1;
                sweep += static_cast<uint32_t>(tn / V);
                pos = tn % V;
                if (sweep >= total_sweeps) {
                    done = true;
                    break;
                }
                if (f >= 0) break;
            }
            if (dcl == 0) {
                c.st[4] += 1;
                if (done) {
                    if (a.rounds_out) a.rounds_out[ch] = c.st[4];
                    const int64_t nxt = ch + stride;
                    init_chain(nxt < a.total_chains ? nxt : -1);
                } else {
                    c.st[1] = pos;
                    c.st[2] = sweep;
                    c.st[3] = emitted;
                }
            }
        }
        chain_sync<WPC>();
    }
}

// ---------------------------------------------------------------------------
// launch wrappers (called by the host runtime)
// ---------------------------------------------------------------------------

// Library-owned scratch of ac_eval_batch_static: the fixed weights and the
// per-workgroup node rows that ac_eval_batch takes from the caller's
// workspace.  One copy per device, alive until the process ends.  On the host
// the name is only a stand-in for the symbol: host code uses the address that
// static_scratch_address returns for the current device, never the name.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

// Device address of this device's copy of `scratch` (call with the device current).
hipError_t static_scratch_address(void **out) {
    return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

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
                       reinterpret_cast<Weight<T> *>(wfix));
    return hipGetLastError();
}

static_assert(sizeof(Weight<float>) == 16 && sizeof(Weight<double>) == 16, "weights are 16 bytes");

// dynamic LDS of the tile kernels: evidence words and angle weights of a tile
size_t lds_bytes(const DevGraph &g) {
    return static_cast<size_t>(g.W) * WAVE * 8 + static_cast<size_t>(g.S_ang) * WAVE * sizeof(Weight<float>);
}

// dynamic LDS of the streaming sampler: evidence words, angle weights and the
// fixed weights, in the pass dtype
template <typename T>
size_t stream_lds_bytes(const DevGraph &g, const SopPlan &sp) {
    return static_cast<size_t>(g.W) * WAVE * 8 + static_cast<size_t>(g.S_ang) * WAVE * sizeof(cplx<T>) +
           static_cast<size_t>(g.S) * sizeof(cplx<T>) + static_cast<size_t>(sp.mask_words) * WAVE * 8;
}

template <typename T>
hipError_t launch_eval(const DevGraph &g, const SopPlan &sp, int grid, int block, const double *theta, const int32_t *param_of, int P,
                       const uint64_t *evidence, int64_t B, const void *wfix, void *vals, size_t per_wg_elems,
                       void *amp_out, double *prob_out, hipStream_t st) {
    size_t lds = lds_bytes(g);
    if (block < WAVE || block > MAX_BLOCK || block % WAVE != 0) return hipErrorInvalidValue;
    auto kern = sp.S > 0 ? k_eval<T, true> : k_eval<T, false>;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, st, g, sp, theta, param_of, P, evidence, B,
                       reinterpret_cast<const Weight<T> *>(wfix), reinterpret_cast<cplx<T> *>(vals),
                       per_wg_elems, reinterpret_cast<cplx<T> *>(amp_out), prob_out);
    return hipGetLastError();
}

size_t mpe_lds_bytes(const DevGraph &g) { return lds_bytes(g) + static_cast<size_t>(g.W) * WAVE * 8; }

hipError_t launch_mpe(const DevGraph &g, const MpePlan &mp, int grid, int block, const double *theta,
                      const int32_t *param_of, int P, const uint64_t *evidence, int64_t B, const void *wfix,
                      void *vals, size_t per_wg_elems, double *prob_out, uint64_t *mpe_out, hipStream_t st) {
    if (block < WAVE || block > MAX_BLOCK || block % WAVE != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mpe, dim3(grid), dim3(block), mpe_lds_bytes(g), st, g, mp, theta, param_of, P, evidence, B,
                       reinterpret_cast<const Weight<double> *>(wfix), reinterpret_cast<cplx<double> *>(vals),
                       per_wg_elems, prob_out, mpe_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_grad(const DevGraph &g, const SopPlan &sp, int grid, int block, const double *theta, const int32_t *param_of,
                       const uint64_t *evidence, int64_t B, const void *wfix, void *vals, size_t per_wg_elems,
                       int mode, const void *cotangent, const double *weight, double *contrib, int P,
                       double *grad, void *amp_out, void *dfdtheta_out, void *dind_out, void *sort_ws,
                       size_t sort_ws_bytes, hipStream_t st) {
    size_t lds = lds_bytes(g);
    if (block < WAVE || block > MAX_BLOCK || block % WAVE != 0) return hipErrorInvalidValue;
    auto kern = sp.S > 0 ? k_grad<T, true> : k_grad<T, false>;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, st, g, sp, theta, param_of, P, evidence, B,
                       reinterpret_cast<const Weight<T> *>(wfix), reinterpret_cast<cplx<T> *>(vals),
                       per_wg_elems, mode, reinterpret_cast<const cplx<T> *>(cotangent), weight, contrib,
                       reinterpret_cast<cplx<T> *>(amp_out), reinterpret_cast<cplx<T> *>(dfdtheta_out),
                       reinterpret_cast<cplx<T> *>(dind_out));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (g.K > 0 && P > 0) {
        uint32_t *keys = reinterpret_cast<uint32_t *>(sort_ws);
        uint32_t *idx = keys + B;
        uint32_t *keys_sorted = idx + B;
        uint32_t *idx_sorted = keys_sorted + B;
        void *tmp = idx_sorted + B;
        const size_t tmp_bytes = sort_ws_bytes - 16 * static_cast<size_t>(B);
        hipLaunchKernelGGL(k_grad_keys, dim3(static_cast<unsigned>((B + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st,
                           param_of, B, P, keys, idx);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        int end_bit = 1;
        while (end_bit < 32 && (static_cast<uint32_t>(P) >> end_bit) != 0u) ++end_bit;   // keys <= P
        size_t need = 0;
        err = hipcub::DeviceRadixSort::SortPairs(nullptr, need, keys, keys_sorted, idx, idx_sorted,
                                                 static_cast<int>(B), 0, end_bit, st);
        if (err != hipSuccess) return err;
        if (need > tmp_bytes) return hipErrorInvalidValue;
        size_t have = tmp_bytes;
        err = hipcub::DeviceRadixSort::SortPairs(tmp, have, keys, keys_sorted, idx, idx_sorted,
                                                 static_cast<int>(B), 0, end_bit, st);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k_grad_segments, dim3(P), dim3(BLOCK), 0, st, keys_sorted, idx_sorted, B, g.K, contrib, grad);
        err = hipGetLastError();
    }
    return err;
}

// Workspace bytes of the gradient reduction's sort for a batch of B elements:
// keys and indices before and after the sort, then the sort's own storage.
size_t grad_sort_bytes(int64_t B) {
    if (B <= 0) return 0;
    size_t tmp = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, static_cast<uint32_t *>(nullptr),
                                           static_cast<uint32_t *>(nullptr), static_cast<uint32_t *>(nullptr),
                                           static_cast<uint32_t *>(nullptr), static_cast<int>(B), 0, 32) != hipSuccess)
        return 0;
    return 16 * static_cast<size_t>(B) + tmp + 256;
}

template <typename T>
hipError_t launch_sample(const DevGraph &g, int grid, const double *theta, const void *wfix, void *vals,
                         size_t per_wg_elems, const SampleArgs &a, hipStream_t st) {
    size_t lds = lds_bytes(g);
    hipLaunchKernelGGL(k_sample<T>, dim3(grid), dim3(BLOCK), lds, st, g, theta,
                       reinterpret_cast<const Weight<T> *>(wfix), reinterpret_cast<cplx<T> *>(vals),
                       per_wg_elems, a);
    return hipGetLastError();
}


template <typename T>
size_t sample_lds_chain_bytes(const DevGraph &g, const LdsPlan &lp) {
    return chain_lds_bytes<T>(lp.N, g.n_ind, g.S, g.n_sel, lp.max_edges, g.W);
}

size_t sample_lds_meta_bytes(const LdsPlan &lp) { return level_meta_bytes(lp.L); }

template <typename T, int CPW, int WPC>
hipError_t launch_sample_lds_cpw(const DevGraph &g, const LdsPlan &lp, int grid, const double *theta,
                                 const double *noise, const SampleArgs &a, hipStream_t st) {
    const uint32_t cb = static_cast<uint32_t>(chain_lds_bytes<T>(lp.N, g.n_ind, g.S, g.n_sel, lp.max_edges, g.W));
    const size_t lds = static_cast<size_t>(cb) * CPW + level_meta_bytes(lp.L);
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sample_lds<T, CPW, WPC>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((k_sample_lds<T, CPW, WPC>), dim3(grid), dim3(WAVE * WPC), lds, st, g, lp, theta, noise, a,
                       cb);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sample_lds(const DevGraph &g, const LdsPlan &lp, int cpw, int wpc, int grid, const double *theta,
                             const double *noise, const SampleArgs &a, hipStream_t st) {
    if (wpc == 4 && cpw == 1) return launch_sample_lds_cpw<T, 1, 4>(g, lp, grid, theta, noise, a, st);
    if (wpc != 1) return hipErrorInvalidValue;
    switch (cpw) {
        case 1: return launch_sample_lds_cpw<T, 1, 1>(g, lp, grid, theta, noise, a, st);
        case 2: return launch_sample_lds_cpw<T, 2, 1>(g, lp, grid, theta, noise, a, st);
        case 4: return launch_sample_lds_cpw<T, 4, 1>(g, lp, grid, theta, noise, a, st);
        default: return hipErrorInvalidValue;
    }
}

// Workgroups of one kernel that fit on a compute unit at once (registers,
// LDS and wave slots), for grids of exactly the co-resident size.
// which: 0 = k_eval, 1 = k_grad, 2 = k_sample, 3 = k_sample_stream; block =
// threads per workgroup.
template <typename T>
int resident_blocks(const DevGraph &g, const SopPlan &sp, int which, int block) {
    const void *fn = nullptr;
    size_t lds = lds_bytes(g);
    switch (which) {
        case 0: fn = sp.S > 0 ? reinterpret_cast<const void *>(&k_eval<T, true>)
                              : reinterpret_cast<const void *>(&k_eval<T, false>); break;
        case 1: fn = sp.S > 0 ? reinterpret_cast<const void *>(&k_grad<T, true>)
                              : reinterpret_cast<const void *>(&k_grad<T, false>); break;
        case 2: fn = reinterpret_cast<const void *>(&k_sample<T>); break;
        case 3:
            fn = sp.occ_sib3 ? reinterpret_cast<const void *>(&k_sample_stream<T, true>)
                             : reinterpret_cast<const void *>(&k_sample_stream<T, false>);
            lds = stream_lds_bytes<T>(g, sp);
            break;
        default: return 1;
    }
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, block, lds) != hipSuccess || n < 1) return 1;
    return n;
}
template int resident_blocks<float>(const DevGraph &, const SopPlan &, int, int);
template int resident_blocks<double>(const DevGraph &, const SopPlan &, int, int);

template size_t sample_lds_chain_bytes<float>(const DevGraph &, const LdsPlan &);
template size_t sample_lds_chain_bytes<double>(const DevGraph &, const LdsPlan &);
template hipError_t launch_sample_lds<float>(const DevGraph &, const LdsPlan &, int, int, int, const double *,
                                             const double *, const SampleArgs &, hipStream_t);
template hipError_t launch_sample_lds<double>(const DevGraph &, const LdsPlan &, int, int, int, const double *,
                                              const double *, const SampleArgs &, hipStream_t);


template <typename T>
hipError_t launch_sample_stream(const DevGraph &g, const SopPlan &sp, int grid, int block, const double *theta,
                                const void *wfix, void *vals, size_t per_wg_elems, const SampleArgs &a,
                                hipStream_t st) {
    if (block < WAVE || block > MAX_BLOCK || block % WAVE != 0) return hipErrorInvalidValue;
    size_t lds = stream_lds_bytes<T>(g, sp);
    if (sp.occ_sib3)
        hipLaunchKernelGGL((k_sample_stream<T, true>), dim3(grid), dim3(block), lds, st, g, sp, theta,
                           reinterpret_cast<const Weight<T> *>(wfix), reinterpret_cast<cplx<T> *>(vals), per_wg_elems, a);
    else
        hipLaunchKernelGGL((k_sample_stream<T, false>), dim3(grid), dim3(block), lds, st, g, sp, theta,
                           reinterpret_cast<const Weight<T> *>(wfix), reinterpret_cast<cplx<T> *>(vals), per_wg_elems, a);
    return hipGetLastError();
}
template hipError_t launch_fixed_slots<float>(const DevGraph &, const double *, void *, hipStream_t);
template hipError_t launch_fixed_slots<double>(const DevGraph &, const double *, void *, hipStream_t);
template hipError_t launch_sample_stream<float>(const DevGraph &, const SopPlan &, int, int, const double *,
                                                const void *, void *, size_t, const SampleArgs &, hipStream_t);
template hipError_t launch_sample_stream<double>(const DevGraph &, const SopPlan &, int, int, const double *,
                                                 const void *, void *, size_t, const SampleArgs &, hipStream_t);

template hipError_t launch_eval<float>(const DevGraph &, const SopPlan &, int, int, const double *, const int32_t *, int, const uint64_t *,
                                       int64_t, const void *, void *, size_t, void *, double *, hipStream_t);
template hipError_t launch_eval<double>(const DevGraph &, const SopPlan &, int, int, const double *, const int32_t *, int, const uint64_t *,
                                        int64_t, const void *, void *, size_t, void *, double *, hipStream_t);
template hipError_t launch_grad<float>(const DevGraph &, const SopPlan &, int, int, const double *, const int32_t *, const uint64_t *,
                                       int64_t, const void *, void *, size_t, int, const void *, const double *,
                                       double *, int, double *, void *, void *, void *, void *, size_t, hipStream_t);
template hipError_t launch_grad<double>(const DevGraph &, const SopPlan &, int, int, const double *, const int32_t *, const uint64_t *,
                                        int64_t, const void *, void *, size_t, int, const void *, const double *,
                                        double *, int, double *, void *, void *, void *, void *, size_t, hipStream_t);
template hipError_t launch_sample<float>(const DevGraph &, int, const double *, const void *, void *, size_t,
                                         const SampleArgs &, hipStream_t);
template hipError_t launch_sample<double>(const DevGraph &, int, const double *, const void *, void *, size_t,
                                          const SampleArgs &, hipStream_t);

}  // namespace qkc
