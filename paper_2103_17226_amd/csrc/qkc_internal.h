// Internal declarations shared by the host runtime and the HIP kernels of
// the AC evaluation library.  Not part of the public C ABI (include/qkc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qkc {

constexpr int WAVE = 64;              // wavefront width on CDNA
constexpr int BLOCK = 256;            // threads per workgroup (4 waves)
constexpr int MAX_BLOCK = 1024;       // tile kernels and streaming sampler: up to 16 waves on one tile
constexpr int MAX_WORDS = 64;         // evidence words staged in LDS
constexpr int MAX_ANGLE_SLOTS = 64;   // angle-dependent weights per element
constexpr int MAX_ANGLES = 64;        // columns of theta
constexpr int MAX_DOM = 16;           // values per evidence variable
constexpr size_t STATIC_SCRATCH_BYTES = size_t{256} << 20;   // scratch of ac_eval_batch_static per device

// child-reference tags (bits 31..30)
constexpr uint32_t TAG_NODE = 0u;
constexpr uint32_t TAG_IND = 1u;
constexpr uint32_t TAG_SLOT = 2u;
constexpr uint32_t TAG_SEL = 3u;      // selector leaf: sum_u lambda_{v=u} W[slot_u]
constexpr uint32_t REF_MASK = 0x3fffffffu;
constexpr uint32_t NO_SLOT = 0xFFFFFFFFu;
constexpr int SEL_DOM = 4;            // values per selector variable
constexpr int SEL_REC = 8;            // u32 per device selector record

// Device encoding of an indicator reference, rewritten at load time so that
// the kernels decode it without table lookups:
//   bits 31..30 tag (1), 29..26 value u, 25..24 field width - 1,
//   23..6 word index, 5..0 bit shift within the word.
__host__ __device__ inline uint32_t dev_ind_ref(uint32_t u, uint32_t width, uint32_t word,
                                                uint32_t shift) {
    return (TAG_IND << 30) | (u << 26) | ((width - 1u) << 24) | (word << 6) | shift;
}

// slot base kinds (see include/qkc.h)
enum SlotBase : uint8_t {
    B_CONST = 0, B_COS = 1, B_SIN = 2, B_EXPM = 3, B_EXPP = 4,
    B_SQRT_1MP = 5, B_SQRT_P3 = 6, B_SQRT_P = 7
};

struct SlotDesc {
    uint8_t base;
    uint8_t coef;      // 0: 1, 1: -1, 2: i, 3: -i
    uint16_t pad;
    int32_t index;
    double scale;
    double re, im;
};
static_assert(sizeof(SlotDesc) == 32, "slot layout");

// Device-resident graph (all pointers into one device allocation).
struct DevGraph {
    const uint8_t *op;          // [N]
    const uint32_t *row_ptr;    // [N+1]
    const uint32_t *col;        // [E] device-encoded refs
    const uint32_t *level_ptr;  // [L+1]
    const SlotDesc *slots;      // [S]
    const uint32_t *par_ptr;    // [N+1]   parent edges of each internal node
    const uint32_t *par_edge;   // [E_node]
    const uint32_t *edge_parent;// [E]
    const uint32_t *leaf_ptr;   // [n_ind + S + 1] parent edges of each leaf
    const uint32_t *leaf_edge;  // [E_leaf]
    const uint32_t *var_field;  // [n_vars] word<<8 | shift<<2 | (width-1)
    const uint32_t *ind_base;   // [n_vars+1]
    const double *noise_default;// [n_noise]
    const uint32_t *sel;        // [SEL_REC * n_sel] field (word<<8|shift<<2|width-1), slot[4], pad
    const uint32_t *vsel_ptr;   // [n_vars+1] selectors of each variable
    const uint32_t *vsel;       // [n_sel]
    const uint64_t *par_rec;    // [E_node] parent | sibling << 32 of each par_edge entry
    const uint64_t *leaf_rec;   // [E_leaf] the same for each leaf_edge entry
    int32_t N, L, root, S, S_ang, n_vars, W, n_ind, K, n_noise, n_qubits, n_sel;
    int64_t E;
};

// Node-parallel plan of the DAG, derived at load time for the LDS-resident
// kernels.  Every node has at most two children: k-ary products become
// chains and k-ary sums balanced trees of binary nodes.  Nodes are levelled
// as soon as possible and, within a level, sums come before products.
//   fwd[i]        children refs a | b << 32 (b = IDENT_REF for a single child)
//   level_prod[l] first product of level l (sums are [level_ptr[l], level_prod[l]))
//   brec[t]       for node t < N, indicator leaf t - N < n_ind or selector
//                 vsel[t - N - n_ind] (selector targets follow the
//                 per-variable selector lists): {number of parent
//                 edges, offset of the 2nd.. in orec, first parent, first
//                 sibling}; a parent edge contributes adj[parent] * value(sibling),
//                 sibling = NO_SIBLING for a sum parent
//   orec[q]       further parent edges: parent | sibling << 32
constexpr uint32_t NO_SIBLING = 0xFFFFFFFFu;
constexpr uint32_t IDENT_REF = 0xFFFFFFFFu;
// sibling field of a parent-edge record whose parent is a product of three or
// more children (the other children's product is formed on the fly)
constexpr uint32_t MULTI_SIBLING = 0xFFFFFFFEu;

//   estart[t]     the same parent edges as one CSR sorted by target t:
//   edg[e]        edges [estart[t], estart[t+1]) of target t, parent | sibling << 32;
//                 the edges of one level's nodes are contiguous
// The LDS-resident kernel keeps node values, weights and selector values in
// one array [N | S | n_sel]; fwd_u and edg_u are fwd and edg with every
// non-indicator reference rewritten to its index in that array (tag 0), so
// a child is one LDS load whatever its kind.
//   dstart[t], dterm[j]  d root / d lambda for indicator t: the sum over j in
//                 [dstart[t], dstart[t+1]) of leafterm[j & 0xffffffff] *
//                 W[j >> 32] (W index 0xffffffff: factor 1), where leafterm[e]
//                 is the term of leaf edge estart[N] + e
struct LdsPlan {
    const uint64_t *fwd;        // [N]
    const uint32_t *level_ptr;  // [L+1]
    const uint32_t *level_prod; // [L]
    const uint32_t *brec;       // [4 * (N + n_ind + n_sel)]
    const uint64_t *orec;       // [R]
    const uint32_t *estart;     // [N + n_ind + n_sel + 1]
    const uint64_t *edg;        // [estart[N + n_ind + n_sel]]
    const uint64_t *fwd_u;      // [N]
    const uint64_t *edg_u;      // [estart[N + n_ind + n_sel]]
    const uint32_t *dstart;     // [n_ind + 1]
    const uint64_t *dterm;      // [dstart[n_ind]]
    const uint32_t *esel;       // [estart[N + n_ind + n_sel] - estart[N + n_ind]] selector of each selector parent edge
    int32_t N, L, root;
    int32_t max_edges;          // most parent edges of one level, or of all leaves
    int64_t R;
};

// Sum-of-products plan of the DAG, derived at load time for the streaming
// sampler and the upward pass.  Every product node whose only parent is a sum
// is folded into that sum as one of its terms, so a super-node is
//   value = sum over its terms t of (product over the factors f of t)
// where a factor is a leaf or another super-node; a term holds at most
// SOP_MAX_FACTORS factors (a longer product is split into product
// super-nodes, multiplied in the same order).  Folded products never get a
// row of their own: their values stay in registers.  Super-nodes are levelled
// as soon as possible and sorted by level.
//   level_ptr[l]  super-nodes of level l are [level_ptr[l], level_ptr[l+1])
//   fptr[s]       factors of super-node s are [fptr[s], fptr[s+1]), term by term
//   frec[f]       factor reference (tag 0: super-node index; leaves as in the
//                 device graph) | SOP_LAST_OF_TERM if it ends its term
//                 | SOP_DIRECT if the term is a sum's child that is not a product
//   ostart[t]     occurrences of target t as a factor: super-node t < S,
//                 indicator leaf S + i, selector S + n_ind + k with the
//                 selectors in per-variable order (vsel), angle-dependent
//                 weight slot S + n_ind + n_sel + s
//   occ[4 o ..]   {parent super-node, three sibling references}: the
//                 occurrence contributes adj[parent] times the product of its
//                 siblings (the other factors of its term; NO_SIBLING pads)
//   osel[o - ostart[S + n_ind]]  selector of each selector occurrence
constexpr int SOP_MAX_FACTORS = 4;
constexpr uint64_t SOP_LAST_OF_TERM = 1ull << 32;
// a term that is a sum's own child (not a folded product): its one factor is
// added as it is rather than multiplied into a product
constexpr uint64_t SOP_DIRECT = 1ull << 33;
struct SopPlan {
    const uint32_t *level_ptr;  // [L+1]
    const uint32_t *fptr;       // [S+1]
    const uint64_t *frec;       // [fptr[S]]
    const uint32_t *ostart;     // [S + n_ind + n_sel + S_ang + 1]
    const uint32_t *occ;        // [4 * ostart[S + n_ind + n_sel + S_ang]]
    const uint32_t *osel;       // [selector occurrences]
    int32_t S, L, root;
    int32_t max_factors;        // most factors of one super-node
    int32_t mask_words;         // words of the per-chain change mask of the streaming
                                // sampler's decision pass (0: decisions in the scan only)
    int32_t occ_sib3;           // 1 if an occurrence of a super-node or an indicator or
                                // selector leaf has three siblings (the streaming
                                // passes then walk occurrences in smaller groups)
    // Row reuse for the upward pass alone (no downward pass reads the values
    // later): a super-node's row is free once its last consumer's level has
    // run, so rows are handed out again level by level (greedy in level order,
    // which needs exactly the largest number of super-nodes alive at once).
    const uint64_t *frec_live;  // frec with super-node references replaced by their rows
    const uint32_t *srow;       // [S] row of each super-node
    int32_t live_rows;          // rows the upward pass needs per element
};
constexpr int MAX_MASK_WORDS = 16;   // decision pass for up to 1024 variables

// Most-probable-explanation queries: big[i] = 1 for the nodes with a
// noise-event indicator below them (their rows hold max-products of
// squared magnitudes), event_mask[w] = bits of word w that hold noise-event
// fields.
struct MpePlan {
    const uint8_t *big;         // [N]
    const uint64_t *event_mask; // [W]
    int32_t n_qubits;
};

// Arguments of the Gibbs sampler kernel.
struct SampleArgs {
    int64_t total_chains;
    int32_t cpp, spc, burn_in, thin;
    uint64_t seed;
    int32_t n_cost_edges;
    const int32_t *cost_edges;
    uint64_t *samples;
    uint64_t *states_out;
    double *cost_out;
    int64_t *rounds_out;
    int32_t nwq;
    const uint64_t *init_states;   // [total_chains][W] start states, or null for the seeded start
    uint64_t first_sweep;          // RNG sweep number of this call's first sweep
    int32_t first_var;             // the scan visits variables first_var .. n_vars-1
    int32_t seq_scan;              // 1: every visit decided in the scan (no decision pass)
    uint64_t chain_offset;         // RNG chain number of this call's chain 0
};

}  // namespace qkc
