// Host-only stand-ins for the library's device-side functions, so that the
// planner and the cost model's host code can be built and run alone under
// AddressSanitizer / UndefinedBehaviorSanitizer.  Nothing here runs a kernel:
// every run entry point reports that this build has no device.
#include "fz_internal.h"
#include "generic.h"

namespace fz {
const int JIT_TILES[N_JIT_TILES][2] = {{16, 16}, {32, 16}, {32, 32}, {64, 16}, {64, 32}};
fz_status run_plan(const fz_plan&, const void*, void*, fz_point*, uint32_t*, uint32_t, void*, size_t, void*)
{
    return fail(FZ_E_UNSUPPORTED, "host-only build");
}
size_t workspace_bytes(const fz_plan&) { return 0; }
size_t measure_workspace_bytes(const fz_plan&) { return 0; }
fz_status plan_measure(fz_plan&, const void*, void*, size_t, int, void*)
{
    return fail(FZ_E_UNSUPPORTED, "host-only build");
}
fz_status run_batch(fz_plan&, const fz_clip*, int, void*, size_t, void*)
{
    return fail(FZ_E_UNSUPPORTED, "host-only build");
}
size_t batch_workspace_bytes(const fz_plan&, const fz_clip*, int) { return 0; }
void release_batch(fz_plan&) {}
fz_status jit_prepare(const fz_plan&, const Segment&) { return FZ_OK; }
}  // namespace fz
