// Chunked execution engine (Section III-D of the paper: query free device
// memory, reserve a fixed fraction of it, size the chunks so each fits with
// its padding, run the chunks independently on one GPU).
#pragma once

#include <vector>

#include "common.h"

namespace harpia {

// One filter step of a pipeline.
struct Stage {
    enum Kind { GAUSS, MORPH, MORPH_BOTH, EDGE, THRESH } kind;
    harpia_dtype in_t, out_t;  // element types read and written by the step
    int r[3];                  // radius per axis (the halo this step needs)
    GaussTaps taps;            // GAUSS
    MorphSpec morph;           // MORPH / MORPH_BOTH
    int edge;                  // EDGE: harpia_edge (Sobel / Prewitt)
    int thr_method;            // THRESH: harpia_threshold_method (weights in taps)
    float thr_k, thr_r, thr_offset;
};

struct Job {
    const void *in;
    void *out;
    void *out2;  // second output of MORPH_BOTH (same dtype as out)
    int64_t n[3];
    std::vector<Stage> stages;
    const harpia_exec *ex;
};

// Byte cost of one chunk's buffer set, for the planner.
struct ChunkCost {
    bool host;              // staging buffers for host-resident volumes
    size_t in_es, out_es;   // element sizes of the staged input / output
    int n_out;              // outputs per voxel (2 for MORPH_BOTH)
    const std::vector<Stage> *stages;
};

size_t chunk_bytes(const ChunkCost &c, const int64_t core[3], const int64_t n[3]);

// Plan the tiling of n[] into cores with halo[] per side within `budget`
// bytes (Section III-D, step 2).  chunk[] = {0,0,0} picks z-slabs: the
// deepest slab (full y and x) that fits, capped so that large volumes give
// several chunks to overlap transfers with compute.  Throws on failure.
void plan_chunks(const int64_t n[3], const int32_t halo[3], const int64_t chunk[3], const ChunkCost &cost,
                 size_t budget, int max_buffers, harpia_plan &p);

// Device budget in bytes (Section III-D, step 1: free device memory is
// queried and a fixed fraction of it is reserved):
//   budget = min(cap, fraction x free), or fraction x free without a cap.
// cap = ex->device_budget_bytes, else HARPIA_DEVICE_BUDGET (bytes) as the
// default of callers that give none; fraction = ex->budget_fraction, else
// HARPIA_BUDGET_FRACTION, else HARPIA_DEFAULT_BUDGET_FRACTION.  Without a
// device (plan-only calls) the cap is returned unclipped.
size_t resolve_budget(const harpia_exec *ex);

// Device memory owned for the duration of one call (freed by the
// destructor).  alloc() honours the HARPIA_TEST_FAIL_ALLOC_AT test hook.
struct DevBuf {
    void *p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    void alloc(size_t bytes);
};

bool is_device_pointer(const void *ptr);
void reset_alloc_counter();

// Run a job: resident on the caller's stream when `in`/`out` are device
// pointers, streamed chunk by chunk when they are host pointers.
void run_job(const Job &job);

}  // namespace harpia
