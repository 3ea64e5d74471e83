// Host-side state of a simulation handle and the helpers shared by the
// forward (api.cpp) and adjoint (api_adj.cpp) drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "tfl_internal.h"

struct tfl_sim {
    tfl_config cfg;
    long long N = 0;
    int esz = 8;
    void *E[3] = {nullptr, nullptr, nullptr};
    void *H[3] = {nullptr, nullptr, nullptr};
    void *J[3] = {nullptr, nullptr, nullptr};
    const void *eps = nullptr, *sig = nullptr, *ell = nullptr;
    void *work = nullptr;
    double *scratch = nullptr;
    void *fused = nullptr;  // second E, H set of the fused sweep (caller-owned), or null
    void *cls = nullptr;    // edge classes and their table (caller-owned), or null: the maps path
    int ncls = 0;
    bool state_bound = false, work_bound = false, maps_bound = false;
    size_t work_bytes = 0;
    // workspace layout (element offsets in units of the field type)
    size_t table_off[3] = {0, 0, 0};   // 6 tables of n[a] entries per CPML axis
    size_t psi_off[3] = {0, 0, 0};     // 4 arrays of slab size per CPML axis
    size_t psi_count[3] = {0, 0, 0};   // elements per auxiliary array
    int64_t step = 0;
    bool sampled0 = false;
    bool probes_dirty = true;  // descriptors not yet uploaded to scratch
    std::vector<tfl::SourceDesc> src;
    std::vector<tfl::ProbeDesc> probe;
    double max_ell = 0.0;
    // last tfl_forward_checkpointed run; invalidated by anything that changes what a recomputation
    // of it would produce (maps, sources)
    bool ckpt_valid = false;
    int64_t ckpt_n0 = 0, ckpt_nsteps = 0, ckpt_seg = 0;
    tfl_objective ckpt_obj{};
    // non-finite check every check_every steps (0: off); `checking` while an entry point that
    // reports it runs (tfl_step, tfl_forward_checkpointed), `checked` once a check was launched
    int64_t check_every = 0;
    bool checking = false, checked = false;
    // sweep policy (TFL_SWEEP_*) and the steps of the last tfl_step call per path: two passes, fused
    // sweep, two-step sweep
    int sweep = TFL_SWEEP_AUTO;
    int64_t sweep_counts[3] = {0, 0, 0};
    std::string err;
};


namespace tfl {
namespace detail {

int fail(tfl_sim *s, int code, const char *fmt, ...);
int hip_fail(tfl_sim *s, hipError_t e, const char *where);
bool aligned(const void *p);
size_t round256(size_t bytes);
int check_bound(tfl_sim *s, bool need_maps);
bool box_ok(const tfl_config &c, const int64_t *b);
template <typename T> StepArgs<T> make_args(const tfl_sim *s);
// nsteps forward steps; ev (optional) receives 2 nsteps + 1 events; with
// probes = false the probe kernels are skipped (recomputation in the adjoint).
template <typename T> int do_step(tfl_sim *s, int64_t nsteps, hipStream_t st, hipEvent_t *ev = nullptr,
                                  bool probes = true);
int copy_state(tfl_sim *s, void *dst, const void *src, bool save, hipStream_t st);
// The fused sweep needs periodic boundaries on every axis.
// Layout of the fused sweep's buffer: six field arrays (the second E, H set) of
// the returned stride, then on each CPML axis the second set of its two H-side
// variables at byte offset psi_at[axis]; *total (if given) is the size.
size_t fused_layout(const tfl_sim *s, size_t psi_at[3], size_t *total = nullptr);
// Device pointers of the bound edge classes (x, y, z) and class table; all null when none are bound.
void class_pointers(const tfl_sim *s, const uint16_t *cls[3], const void **table);

// scratch buffer layout: reduction partials, the objective DFT, probe descriptors, and two halves
// for the sweeps' probe copies (a sweep writes one half while it sums the other; a two-step sweep
// writes its two steps' copies to the two quarters of its half)
constexpr size_t kScratchBytes = 1 << 20;
constexpr int kRedBlocks = 1024;            // reductions use doubles [0, 5 * kRedBlocks)
constexpr size_t kObjectiveSlot = 6144;     // doubles [6144, 6146): objective DFT
constexpr size_t kNonfiniteOffset = 49408;  // bytes: two uint64 counters of the non-finite check
constexpr size_t kProbeDescOffset = 65536;  // bytes: TFL_MAX_PROBES + 1 ProbeDesc
constexpr size_t kProbeCopyOffset = 1 << 17;
constexpr size_t kProbeCopyHalf = (kScratchBytes - kProbeCopyOffset) / 2;
static_assert(kNonfiniteOffset >= (kObjectiveSlot + 2) * sizeof(double) && kNonfiniteOffset + 16 <= kProbeDescOffset,
              "non-finite counters overlap the objective or the probe descriptors");
static_assert(kProbeDescOffset + (TFL_MAX_PROBES + 1) * sizeof(ProbeDesc) <= kProbeCopyOffset, "scratch too small");
static_assert(sizeof(AdjArgs<double>) <= 4096 && sizeof(StepArgs<double>) <= 4096 &&
                  sizeof(GradSigmaArgs<double>) <= 4096,
              "kernel arguments above 4 KiB");
// Value soft source d adds at time t (its waveform times its amplitude).
double source_value(const SourceDesc &d, double t);
// Boxes of the bound sources into sd (values zero), and their values at time t.
void source_boxes(const tfl_sim *s, SideArgs &sd);
void source_values(const tfl_sim *s, SideArgs &sd, double t);
// Upload the probe descriptors to scratch when they changed (synchronises).
int upload_probes(tfl_sim *s, hipStream_t st);
// Non-finite check around an entry point's steps: begin clears the counters when the check is on;
// end (after the steps) reads them back when a check ran, synchronising, and fails with
// TFL_E_NONFINITE when any value was found.
int nonfinite_begin(tfl_sim *s, hipStream_t st);
int nonfinite_end(tfl_sim *s, hipStream_t st);

}  // namespace detail
}  // namespace tfl
