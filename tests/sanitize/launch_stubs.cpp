// Stand-ins for the device side of libvk (vk_kernels.hip) so that the host code of vk_api.cpp
// links into a host-only library built with AddressSanitizer and UndefinedBehaviorSanitizer.
// The sanitizer tests drive only calls that never launch (description checks and builders,
// the generated specialisation source, argument errors); any launcher reached aborts.
#include <cstdio>
#include <cstdlib>

#include "vk_launch.hpp"

namespace vk {
namespace {
[[noreturn]] void no_device(const char *what) {
    std::fprintf(stderr, "sanitizer build: %s needs the device code\n", what);
    std::abort();
}
}  // namespace

hipError_t launch_fk_spheres(const RobotDev &, const float *, int64_t, int64_t, float *, int64_t,
                             hipStream_t) { no_device("launch_fk_spheres"); }
int states_split(const RobotDev &, int64_t, int, int) { no_device("states_split"); }
size_t states_scratch_bytes(int64_t n) { return 256 + (size_t)n * 4; }
hipError_t launch_validate_states(const RobotDev &, const EnvDev &, const float *, int64_t, int64_t,
                                  uint8_t *, int, void *, hipStream_t, const StepRanges *) {
    no_device("launch_validate_states");
}
int64_t noalloc_max_states() { return int64_t(1) << 22; }
hipError_t noalloc_scratch(void **) { no_device("noalloc_scratch"); }
hipError_t launch_reset_queue(unsigned long long *, hipStream_t, uint8_t *, int64_t) {
    no_device("launch_reset_queue");
}
hipError_t launch_shortcut_propose(const int32_t *, int64_t, int, int, const uint32_t *, int32_t *,
                                  hipStream_t) { no_device("launch_shortcut_propose"); }
hipError_t launch_shortcut_apply(float *, int32_t *, int64_t, int, int, int, const int32_t *,
                                const uint8_t *, uint8_t *, hipStream_t) {
    no_device("launch_shortcut_apply");
}
hipError_t launch_validate_edges(const RobotDev &, const EnvDev &, const EdgeSrc &, int64_t, float,
                                 uint8_t *, unsigned long long *, int, int, int, int, int,
                                 hipStream_t, unsigned long long *) { no_device("launch_validate_edges"); }
hipError_t launch_validate_edges_spec(const SpecEdgeKernels &, const RobotDev &, const EnvDev &,
                                      const EdgeSrc &, int64_t, float, uint8_t *,
                                      unsigned long long *, int, int, int, int, int, hipStream_t,
                                      unsigned long long *) {
    no_device("launch_validate_edges_spec");
}
hipError_t launch_validate_edge_one(const RobotDev &, const EnvDev &, const EdgeSrc &, int64_t, float,
                                    uint8_t *, hipStream_t) { no_device("launch_validate_edge_one"); }
int knn_parts(int64_t) { no_device("knn_parts"); }
size_t knn_workspace_bytes(int64_t, int) { no_device("knn_workspace_bytes"); }
size_t knn_workspace_bound(int64_t, int) { no_device("knn_workspace_bound"); }
hipError_t launch_knn(const float *, int64_t, int, int, int32_t *, float *, void *, hipStream_t) {
    no_device("launch_knn");
}
hipError_t launch_knn_pairs(const int32_t *, int64_t, int, int32_t *, hipStream_t) {
    no_device("launch_knn_pairs");
}
hipError_t launch_tree_nearest(const float *, const int32_t *, int, int, int64_t, const float *,
                               const uint8_t *, int32_t *, hipStream_t) { no_device("launch_tree_nearest"); }
hipError_t launch_tree_steer(const float *, int, int, int64_t, const int32_t *, const float *, float,
                             float *, uint8_t *, hipStream_t) { no_device("launch_tree_steer"); }
hipError_t launch_tree_append(float *, int32_t *, int32_t *, int, int, int64_t, const float *,
                              const int32_t *, const uint8_t *, int32_t *, hipStream_t) {
    no_device("launch_tree_append");
}
hipError_t launch_rrt_extend(const float *, const int32_t *, int, int, int64_t, const float *,
                             const uint8_t *, float, float *, float *, int32_t *, uint8_t *,
                             hipStream_t) { no_device("launch_rrt_extend"); }
hipError_t launch_rrt_commit(float *, int32_t *, int32_t *, int, int, int64_t, const float *,
                             const int32_t *, const uint8_t *, const uint8_t *, uint8_t *, int32_t *,
                             const int32_t *, int64_t *, int64_t *, uint8_t *, uint64_t *,
                             hipStream_t) { no_device("launch_rrt_commit"); }
hipError_t launch_cost_fwd(const RobotDev &, const EnvDev &, const float *, int64_t, int64_t,
                           float *, hipStream_t) { no_device("launch_cost_fwd"); }
size_t cost_bwd_slot_bytes(const RobotDev &, int, int) { no_device("cost_bwd_slot_bytes"); }
size_t walk_lds_bytes(const RobotDev &, int, int) { no_device("walk_lds_bytes"); }
int walk_block(const RobotDev &, int) { no_device("walk_block"); }
hipError_t launch_cost_bwd(const RobotDev &, const EnvDev &, const float *, int64_t, int64_t,
                           const float *, float *, int64_t, int, hipStream_t, float *, float *) {
    no_device("launch_cost_bwd");
}
size_t cost_bwd_global_slot_bytes(const RobotDev &, int64_t, int) {
    no_device("cost_bwd_global_slot_bytes");
}
int cost_bwd_lds_waves_per_cu(const RobotDev &, int) { no_device("cost_bwd_lds_waves_per_cu"); }
void fill_node(KernelNode &, unsigned long long *, unsigned long long, int, int) { no_device("fill_node"); }
void edge_batch_node(KernelNode &, const BatchSet *, const int32_t *, int, int64_t, float,
                     unsigned long long *, int, int, int, int, int) { no_device("edge_batch_node"); }
}  // namespace vk
