// Internal declarations shared by the host runtime and the HIP kernels of
// the AC evaluation library.  Not part of the public C ABI (include/qkc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qkc {

constexpr int WAVE = 64;              // wavefront width on CDNA
constexpr int BLOCK = 256;            // threads per workgroup (4 waves)
constexpr int MAX_WORDS = 64;         // evidence words staged in LDS
constexpr int MAX_ANGLE_SLOTS = 64;   // angle-dependent weights per element
constexpr int MAX_ANGLES = 64;        // columns of theta
constexpr int MAX_DOM = 16;           // values per evidence variable

// child-reference tags (bits 31..30)
constexpr uint32_t TAG_NODE = 0u;
constexpr uint32_t TAG_IND = 1u;
constexpr uint32_t TAG_SLOT = 2u;
constexpr uint32_t REF_MASK = 0x3fffffffu;

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
    int32_t N, L, root, S, S_ang, n_vars, W, n_ind, K, n_noise, n_qubits;
    int64_t E;
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
};

}  // namespace qkc
