// spect_internal.h - shared by the host translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

struct spect_plan;

namespace spect_internal {
// Set the thread's spect_last_error() message and return code.
int set_error(int code, const char *msg);
// Clear the message and return SPECT_OK.
int clear_error();

// Iteration-level batching (the server's engine).  One tick advances each
// listed request by one step through the work-list kernels: the
// sensitivity pass of subset `subset` (sens != 0; it also writes that
// subset's attenuation table when mu is given) or the OSEM subiteration on
// subset `subset`.  region: the request's state, tick_region_bytes() bytes
// laid out as osem_reconstruct's workspace (the same arguments and tuning,
// so the result equals osem_reconstruct's bitwise).
struct TickItem {
    const spect_plan *plan;
    float *f;
    const float *mu, *g, *s_add;
    char *region;
    int n_subsets;
    int sens;
    int subset;
    int first_sub;  // the request's first subiteration: copy f into the forward's padded layout first
};
int tick_region_bytes(const spect_plan *p, int n_subsets, bool mu, size_t *bytes);
// Voxel-angles of one subiteration (N^2 Nz times the larger subset size),
// the server's measure of a step's work.
double step_work(const spect_plan *p, int n_subsets);
// Host-side launch tables of one tick (no device work); tick_bytes() is the
// size of the buffers tick_launch needs.
struct TickTables;
TickTables *tick_build(const TickItem *items, int n, int *status);
size_t tick_bytes(const TickTables *t);
// Copy the tables through host (pinned, tick_bytes) to dev (tick_bytes) on
// the upload stream up, record the event uploaded there, and launch the
// tick's kernels on st behind that event.  The copy thus runs beside the
// kernels already queued on st instead of between them.  Both buffers stay
// in use until st has passed the tick.
int tick_launch(TickTables *t, char *host, char *dev, hipStream_t st, hipStream_t up, hipEvent_t uploaded);
void tick_free(TickTables *t);
}  // namespace spect_internal
