// Host-only stand-ins for the device side of the library (the kernels and
// their launch wrappers), so that the host runtime (blob parser, plan
// builders, argument checks) can be built with the host compiler's
// sanitizers and fuzzed on a machine without a GPU.  Nothing here is part
// of the library.
#include <hip/hip_runtime.h>

#include "qkc_internal.h"

namespace qkc {

template <typename T>
hipError_t launch_fixed_slots(const DevGraph &, const double *, void *, hipStream_t) { return hipErrorNoDevice; }
template <typename T>
hipError_t launch_eval(const DevGraph &, const SopPlan &, int, int, const double *, const int32_t *, int,
                       const uint64_t *, int64_t, const void *, void *, size_t, void *, double *, hipStream_t) {
    return hipErrorNoDevice;
}
template <typename T>
hipError_t launch_grad(const DevGraph &, const SopPlan &, int, int, const double *, const int32_t *,
                       const uint64_t *, int64_t, const void *, void *, size_t, int, const void *, const double *,
                       double *, int, double *, void *, void *, void *, void *, size_t, hipStream_t) {
    return hipErrorNoDevice;
}
size_t grad_sort_bytes(int64_t B) { return B > 0 ? 16 * static_cast<size_t>(B) + 256 : 0; }
template <typename T>
hipError_t launch_sample(const DevGraph &, int, const double *, const void *, void *, size_t, const SampleArgs &,
                         hipStream_t) {
    return hipErrorNoDevice;
}
size_t lds_bytes(const DevGraph &) { return 0; }
template <typename T>
size_t sample_lds_chain_bytes(const DevGraph &, const LdsPlan &) { return 0; }
size_t sample_lds_meta_bytes(const LdsPlan &) { return 0; }
template <typename T>
hipError_t launch_sample_stream(const DevGraph &, const SopPlan &, int, int, const double *, const void *, void *,
                                size_t, const SampleArgs &, hipStream_t) {
    return hipErrorNoDevice;
}
template <typename T>
hipError_t launch_sample_lds(const DevGraph &, const LdsPlan &, int, int, int, const double *, const double *,
                             const SampleArgs &, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_zero_f64(double *, int64_t, hipStream_t) { return hipErrorNoDevice; }
size_t mpe_lds_bytes(const DevGraph &) { return 0; }
hipError_t launch_mpe(const DevGraph &, const MpePlan &, int, int, const double *, const int32_t *, int,
                      const uint64_t *, int64_t, const void *, void *, size_t, double *, uint64_t *, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t static_scratch_address(void **) { return hipErrorNoDevice; }
template <typename T>
int resident_blocks(const DevGraph &, const SopPlan &, int, int) { return 1; }

#define QKC_INST(T)                                                                                                \
    template hipError_t launch_fixed_slots<T>(const DevGraph &, const double *, void *, hipStream_t);            \
    template hipError_t launch_eval<T>(const DevGraph &, const SopPlan &, int, int, const double *,               \
                                       const int32_t *, int, const uint64_t *, int64_t, const void *, void *,     \
                                       size_t, void *, double *, hipStream_t);                                    \
    template hipError_t launch_grad<T>(const DevGraph &, const SopPlan &, int, int, const double *,               \
                                       const int32_t *, const uint64_t *, int64_t, const void *, void *, size_t, \
                                       int, const void *, const double *, double *, int, double *, void *,        \
                                       void *, void *, void *, size_t, hipStream_t);                              \
    template hipError_t launch_sample<T>(const DevGraph &, int, const double *, const void *, void *, size_t,     \
                                         const SampleArgs &, hipStream_t);                                        \
    template size_t sample_lds_chain_bytes<T>(const DevGraph &, const LdsPlan &);                                 \
    template hipError_t launch_sample_stream<T>(const DevGraph &, const SopPlan &, int, int, const double *,      \
                                                const void *, void *, size_t, const SampleArgs &, hipStream_t);   \
    template hipError_t launch_sample_lds<T>(const DevGraph &, const LdsPlan &, int, int, int, const double *,    \
                                             const double *, const SampleArgs &, hipStream_t);                    \
    template int resident_blocks<T>(const DevGraph &, const SopPlan &, int, int);
QKC_INST(float)
QKC_INST(double)

}  // namespace qkc
