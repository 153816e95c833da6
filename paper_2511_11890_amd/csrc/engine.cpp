// Chunked execution engine: budget, planner, staging, overlap of host<->device
// copies with compute, and the resident device path.
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <thread>

namespace harpia {

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int64_t vol(const int64_t e[3]) { return e[0] * e[1] * e[2]; }

// [lo, hi) = [c0 - e, c1 + e) clipped to [0, n) per axis.
void expand(const int64_t c0[3], const int64_t c1[3], const int64_t e[3], const int64_t n[3], int64_t lo[3],
            int64_t hi[3])
{
    for (int a = 0; a < 3; ++a) {
        lo[a] = std::max<int64_t>(0, c0[a] - e[a]);
        hi[a] = std::min<int64_t>(n[a], c1[a] + e[a]);
    }
}

// Halo still needed after stage k: sum of the radii of stages k+1.. .
void tail_halo(const std::vector<Stage> &st, size_t k, int64_t h[3])
{
    for (int a = 0; a < 3; ++a) {
        h[a] = 0;
        for (size_t j = k + 1; j < st.size(); ++j) h[a] += st[j].r[a];
    }
}

// ------------------------------------------------------------ allocation

thread_local int t_alloc_count = 0;

}  // namespace

bool injected_failure()
{
    const char *env = std::getenv("HARPIA_TEST_FAIL_ALLOC_AT");
    if (!env || !*env) return false;
    const int at = std::atoi(env);
    return at > 0 && ++t_alloc_count == at;
}

void DevBuf::alloc(size_t bytes)
{
    if (bytes == 0) return;
    if (injected_failure()) fail(HARPIA_ERR_OOM, "device allocation failed (injected)");
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        fail(HARPIA_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
}

bool is_device_pointer(const void *ptr);

namespace {

struct PinBuf {
    void *p = nullptr;
    PinBuf() = default;
    PinBuf(const PinBuf &) = delete;
    PinBuf &operator=(const PinBuf &) = delete;
    ~PinBuf()
    {
        if (p) (void)hipHostFree(p);
    }
    void alloc(size_t bytes)
    {
        if (bytes == 0) return;
        if (injected_failure()) fail(HARPIA_ERR_OOM, "pinned allocation failed (injected)");
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            fail(HARPIA_ERR_OOM, "pinned host allocation of " + std::to_string(bytes) + " bytes failed");
        }
    }
};

struct StreamH {
    hipStream_t s = nullptr;
    StreamH() { check_hip(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate"); }
    StreamH(const StreamH &) = delete;
    StreamH &operator=(const StreamH &) = delete;
    ~StreamH()
    {
        if (s) (void)hipStreamDestroy(s);
    }
};

struct EventH {
    hipEvent_t e = nullptr;
    explicit EventH(bool timing = false)
    {
        check_hip(hipEventCreateWithFlags(&e, timing ? hipEventDefault : hipEventDisableTiming), "hipEventCreate");
    }
    EventH(const EventH &) = delete;
    EventH &operator=(const EventH &) = delete;
    ~EventH()
    {
        if (e) (void)hipEventDestroy(e);
    }
};

enum class Mem { Device, Pinned, Pageable };

}  // namespace

bool is_device_pointer(const void *ptr);

namespace {

Mem classify(const void *p)
{
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof(attr));
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return Mem::Pageable;
    }
    if (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged) return Mem::Device;
    if (attr.type == hipMemoryTypeHost) return Mem::Pinned;
    return Mem::Pageable;
}

// ------------------------------------------------------------ stages

// Region of dense device buffer p covering [lo, hi).
Region dense_region(void *p, const int64_t lo[3], const int64_t hi[3])
{
    Region r;
    r.ptr = p;
    r.sy = hi[2] - lo[2];
    r.sz = (hi[1] - lo[1]) * r.sy;
    for (int a = 0; a < 3; ++a) {
        r.o[a] = lo[a];
        r.e[a] = hi[a] - lo[a];
    }
    return r;
}

// Row pitch, in elements, of a chain's intermediate buffer: rows start on
// 16-byte boundaries (a core plus its halo is rarely a multiple of 16
// bytes), so the next kernels keep their widest aligned loads and stores.
// The padding columns are never written or read.
int64_t inter_pitch(int64_t width, size_t es)
{
    const int64_t q = 16 / (int64_t)es;
    return (width + q - 1) / q * q;
}

// Region of an intermediate buffer p covering [lo, hi), rows inter_pitch
// apart.
Region inter_region(void *p, size_t es, const int64_t lo[3], const int64_t hi[3])
{
    Region r = dense_region(p, lo, hi);
    r.sy = inter_pitch(hi[2] - lo[2], es);
    r.sz = (hi[1] - lo[1]) * r.sy;
    return r;
}

// Region [lo, hi) of a whole volume of extent n stored densely at base.
Region volume_region(const void *base, size_t es, const int64_t n[3], const int64_t lo[3], const int64_t hi[3])
{
    Region r;
    r.sy = n[2];
    r.sz = n[1] * n[2];
    const int64_t off = lo[0] * r.sz + lo[1] * r.sy + lo[2];
    r.ptr = const_cast<char *>(static_cast<const char *>(base)) + off * (int64_t)es;
    for (int a = 0; a < 3; ++a) {
        r.o[a] = lo[a];
        r.e[a] = hi[a] - lo[a];
    }
    return r;
}

size_t stage_scratch(const Stage &st, const int64_t ext[3], const int64_t n[3])
{
    if (st.kind != Stage::GAUSS) return 0;
    const bool fused = gauss_slices_fit(n) && (!st.taps.odd || (st.in_t == HARPIA_F32 && st.out_t == HARPIA_F32));
    return gaussian_scratch_bytes(ext, st.r, fused);
}

void launch_stage(const Stage &st, const Region &in, const Region &out, const Region *out2, const int64_t n[3],
                  hipStream_t s, void *scratch, size_t scratch_bytes)
{
    const ChunkArgs a = make_chunk_args(in, out, n);
    bool ok = false;
    switch (st.kind) {
    case Stage::GAUSS: ok = launch_gaussian(a, st.in_t, st.out_t, st.taps, s, scratch, scratch_bytes); break;
    case Stage::MORPH: ok = launch_morph_ex(a, st.in_t, st.morph, false, nullptr, s); break;
    case Stage::MORPH_BOTH: ok = launch_morph_ex(a, st.in_t, st.morph, true, out2, s); break;
    case Stage::EDGE: ok = launch_edge(a, st.in_t, st.out_t, st.edge, s); break;
    case Stage::THRESH:
        ok = launch_local_threshold(a, st.in_t, st.taps, st.thr_method, st.thr_k, st.thr_r, st.thr_offset, s);
        break;
    }
    if (!ok) fail(HARPIA_ERR_UNSUPPORTED, "no kernel for this dtype / radius combination");
    check_hip(hipGetLastError(), "kernel launch");
}

// Run every stage of a chunk whose core is [c0, c1).  `in` covers the
// chunk's input region (or the whole volume); intermediates live in
// `inter` (one dense buffer per stage but the last) and `scratch`.
void run_chunk_stages(const Job &job, const Region &in, const Region &out, const Region *out2,
                      const int64_t c0[3], const int64_t c1[3], void *const *inter, void *scratch,
                      size_t scratch_bytes, hipStream_t s)
{
    Region cur = in;
    for (size_t k = 0; k < job.stages.size(); ++k) {
        const Stage &st = job.stages[k];
        if (k + 1 == job.stages.size()) {
            launch_stage(st, cur, out, out2, job.n, s, scratch, scratch_bytes);
        } else {
            int64_t h[3], lo[3], hi[3];
            tail_halo(job.stages, k, h);
            expand(c0, c1, h, job.n, lo, hi);
            const Region mid = inter_region(inter[k], dtype_size(st.out_t), lo, hi);
            launch_stage(st, cur, mid, nullptr, job.n, s, scratch, scratch_bytes);
            cur = mid;
        }
    }
}

// Device bytes of the intermediates and the largest scratch of a chunk.
void chunk_layout(const std::vector<Stage> &st, const int64_t c0[3], const int64_t c1[3], const int64_t n[3],
                  std::vector<size_t> &inter_bytes, size_t &scratch)
{
    inter_bytes.assign(st.size(), 0);
    scratch = 0;
    for (size_t k = 0; k < st.size(); ++k) {
        int64_t h[3], lo[3], hi[3], ext[3];
        tail_halo(st, k, h);
        expand(c0, c1, h, n, lo, hi);
        for (int a = 0; a < 3; ++a) ext[a] = hi[a] - lo[a];
        if (k + 1 < st.size()) {
            const size_t es = dtype_size(st[k].out_t);
            inter_bytes[k] = align_up((size_t)(ext[0] * ext[1] * inter_pitch(ext[2], es)) * es);
        }
        scratch = std::max(scratch, align_up(stage_scratch(st[k], ext, n)));
    }
}

// Upper bound of chunk_layout over every position of a core of extent
// core[] (an interior chunk's halos are not clipped by a face).
void worst_layout(const std::vector<Stage> &st, const int64_t core[3], const int64_t n[3],
                  std::vector<size_t> &inter_bytes, size_t &scratch)
{
    inter_bytes.assign(st.size(), 0);
    scratch = 0;
    for (size_t k = 0; k < st.size(); ++k) {
        int64_t h[3], ext[3];
        tail_halo(st, k, h);
        for (int a = 0; a < 3; ++a) ext[a] = std::min(n[a], std::min(core[a], n[a]) + 2 * h[a]);
        if (k + 1 < st.size()) {
            const size_t es = dtype_size(st[k].out_t);
            inter_bytes[k] = align_up((size_t)(ext[0] * ext[1] * inter_pitch(ext[2], es)) * es);
        }
        scratch = std::max(scratch, align_up(stage_scratch(st[k], ext, n)));
    }
}

// ------------------------------------------------------------ host copies

struct Copy3D {
    // Copy the box [lo, hi) between a host volume (extent n) and a dense
    // device buffer.
    static void run(bool h2d, void *host, size_t es, const int64_t n[3], const int64_t lo[3], const int64_t hi[3],
                    void *dev, hipStream_t s)
    {
        const int64_t ex = hi[2] - lo[2], ey = hi[1] - lo[1], ez = hi[0] - lo[0];
        char *hbase = static_cast<char *>(host) + ((lo[0] * n[1] + lo[1]) * n[2] + lo[2]) * (int64_t)es;
        if (ex == n[2] && ey == n[1]) {  // contiguous slab
            const size_t bytes = (size_t)(ez * ey * ex) * es;
            check_hip(h2d ? hipMemcpyAsync(dev, hbase, bytes, hipMemcpyHostToDevice, s)
                          : hipMemcpyAsync(hbase, dev, bytes, hipMemcpyDeviceToHost, s),
                      "hipMemcpyAsync");
            return;
        }
        if (ex == n[2]) {  // each z-slice of the box is contiguous
            const size_t w = (size_t)(ey * ex) * es, hp = (size_t)(n[1] * n[2]) * es;
            check_hip(h2d ? hipMemcpy2DAsync(dev, w, hbase, hp, w, (size_t)ez, hipMemcpyHostToDevice, s)
                          : hipMemcpy2DAsync(hbase, hp, dev, w, w, (size_t)ez, hipMemcpyDeviceToHost, s),
                      "hipMemcpy2DAsync");
            return;
        }
        hipMemcpy3DParms p;
        std::memset(&p, 0, sizeof(p));
        const hipPitchedPtr hp =
            make_hipPitchedPtr(host, (size_t)n[2] * es, (size_t)n[2], (size_t)n[1]);
        const hipPitchedPtr dp = make_hipPitchedPtr(dev, (size_t)ex * es, (size_t)ex, (size_t)ey);
        const hipPos hpos = make_hipPos((size_t)lo[2] * es, (size_t)lo[1], (size_t)lo[0]);
        const hipPos zero = make_hipPos(0, 0, 0);
        p.extent = make_hipExtent((size_t)ex * es, (size_t)ey, (size_t)ez);
        if (h2d) {
            p.srcPtr = hp;
            p.srcPos = hpos;
            p.dstPtr = dp;
            p.dstPos = zero;
            p.kind = hipMemcpyHostToDevice;
        } else {
            p.srcPtr = dp;
            p.srcPos = zero;
            p.dstPtr = hp;
            p.dstPos = hpos;
            p.kind = hipMemcpyDeviceToHost;
        }
        check_hip(hipMemcpy3DAsync(&p, s), "hipMemcpy3DAsync");
    }
};

// Host-side gather / scatter between a pageable host volume and a dense
// pinned staging buffer, split over a few threads.
void host_box_copy(bool to_dense, void *host, size_t es, const int64_t n[3], const int64_t lo[3],
                   const int64_t hi[3], void *dense)
{
    const int64_t ex = hi[2] - lo[2], ey = hi[1] - lo[1], ez = hi[0] - lo[0];
    const int64_t rows = ez * ey;
    const size_t rb = (size_t)ex * es;
    auto work = [&](int64_t r0, int64_t r1) {
        for (int64_t r = r0; r < r1; ++r) {
            const int64_t z = lo[0] + r / ey, y = lo[1] + r % ey;
            char *hp = static_cast<char *>(host) + ((z * n[1] + y) * n[2] + lo[2]) * (int64_t)es;
            char *dp = static_cast<char *>(dense) + (size_t)r * rb;
            if (to_dense)
                std::memcpy(dp, hp, rb);
            else
                std::memcpy(hp, dp, rb);
        }
    };
    const int64_t bytes = rows * (int64_t)rb;
    int nt = bytes > (64 << 20) ? 8 : 1;
    if (nt == 1) {
        work(0, rows);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(work, rows * t / nt, rows * (t + 1) / nt);
    for (auto &t : th) t.join();
}

void chunk_box(const harpia_plan &p, int64_t i, int64_t c0[3], int64_t c1[3])
{
    const int64_t gx = p.grid[2], gy = p.grid[1];
    const int64_t idx[3] = {i / (gx * gy), (i / gx) % gy, i % gx};
    for (int a = 0; a < 3; ++a) {
        c0[a] = idx[a] * p.core[a];
        c1[a] = std::min(p.shape[a], c0[a] + p.core[a]);
    }
}

int32_t total_halo(const std::vector<Stage> &st, int a)
{
    int32_t h = 0;
    for (const Stage &s : st) h += s.r[a];
    return h;
}

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ------------------------------------------------------------ device path

void run_device(const Job &job, harpia_stats *stats)
{
    const harpia_exec *ex = job.ex;
    hipStream_t s = ex ? static_cast<hipStream_t>(ex->stream) : nullptr;
    const bool force = ex && (ex->flags & HARPIA_F_FORCE_CHUNKED);
    const Stage &first = job.stages.front();
    const Stage &last = job.stages.back();
    const size_t in_es = dtype_size(first.in_t), out_es = dtype_size(last.out_t);
    const int64_t zero[3] = {0, 0, 0};
    const Region vin = volume_region(job.in, in_es, job.n, zero, job.n);

    std::vector<size_t> inter;
    size_t scratch = 0;
    chunk_layout(job.stages, zero, job.n, job.n, inter, scratch);
    size_t whole = scratch;
    for (size_t b : inter) whole += b;

    if (!force && whole == 0) {  // one fused launch, asynchronous on s
        const Region vout = volume_region(job.out, out_es, job.n, zero, job.n);
        Region vout2;
        if (job.out2) vout2 = volume_region(job.out2, out_es, job.n, zero, job.n);
        run_chunk_stages(job, vin, vout, job.out2 ? &vout2 : nullptr, zero, job.n, nullptr, nullptr, 0, s);
        if (stats) {
            stats->n_chunks = 1;
            stats->peak_device_bytes = 0;
        }
        return;
    }

    const size_t budget = resolve_budget(ex);
    harpia_plan p;
    ChunkCost cost{false, in_es, out_es, job.out2 ? 2 : 1, &job.stages};
    int32_t halo[3] = {total_halo(job.stages, 0), total_halo(job.stages, 1), total_halo(job.stages, 2)};
    if (!force && whole <= budget) {
        p.core[0] = job.n[0];
        p.core[1] = job.n[1];
        p.core[2] = job.n[2];
        for (int a = 0; a < 3; ++a) {
            p.shape[a] = job.n[a];
            p.grid[a] = 1;
            p.halo[a] = halo[a];
        }
        p.n_chunks = 1;
        p.n_buffers = 1;
        p.device_bytes = whole;
        p.budget_bytes = budget;
    } else {
        plan_chunks(job.n, halo, ex ? ex->chunk : zero, cost, budget, 1, p);
    }

    // Arena sized for the largest chunk (an interior full core).
    int64_t c0[3], c1[3];
    worst_layout(job.stages, p.core, job.n, inter, scratch);
    size_t arena_bytes = scratch;
    for (size_t b : inter) arena_bytes += b;
    DevBuf arena;
    arena.alloc(arena_bytes);
    std::vector<void *> inter_ptr(job.stages.size(), nullptr);
    char *cursor = static_cast<char *>(arena.p);
    for (size_t k = 0; k < inter.size(); ++k) {
        inter_ptr[k] = cursor;
        cursor += inter[k];
    }
    void *scratch_ptr = scratch ? cursor : nullptr;

    for (int64_t i = 0; i < p.n_chunks; ++i) {
        chunk_box(p, i, c0, c1);
        const Region vout = volume_region(job.out, out_es, job.n, c0, c1);
        Region vout2;
        if (job.out2) vout2 = volume_region(job.out2, out_es, job.n, c0, c1);
        run_chunk_stages(job, vin, vout, job.out2 ? &vout2 : nullptr, c0, c1, inter_ptr.data(), scratch_ptr,
                         scratch, s);
    }
    // The arena is released before returning: wait for the work that uses it.
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (stats) {
        stats->n_chunks = p.n_chunks;
        stats->peak_device_bytes = (int64_t)arena_bytes;
        stats->budget_bytes = (int64_t)budget;
    }
}

// ------------------------------------------------------------ host path

void run_host(const Job &job, Mem min, Mem mout, harpia_stats *stats)
{
    const harpia_exec *ex = job.ex;
    const Stage &first = job.stages.front();
    const Stage &last = job.stages.back();
    const size_t in_es = dtype_size(first.in_t), out_es = dtype_size(last.out_t);
    const int n_out = job.out2 ? 2 : 1;
    const size_t budget = resolve_budget(ex);
    int32_t halo[3] = {total_halo(job.stages, 0), total_halo(job.stages, 1), total_halo(job.stages, 2)};
    const int64_t zero[3] = {0, 0, 0};
    ChunkCost cost{true, in_es, out_es, n_out, &job.stages};
    harpia_plan p;
    plan_chunks(job.n, halo, ex ? ex->chunk : zero, cost, budget, 3, p);
    const int NB = p.n_buffers;

    // Per buffer set: staged input, staged output(s), intermediates, scratch.
    int64_t c0[3], c1[3], lo[3], hi[3];
    int64_t hh[3] = {halo[0], halo[1], halo[2]};
    int64_t iext[3], cext[3];
    for (int a = 0; a < 3; ++a) {
        iext[a] = std::min(job.n[a], p.core[a] + 2 * hh[a]);
        cext[a] = p.core[a];
    }
    const size_t in_bytes = align_up((size_t)vol(iext) * in_es);
    const size_t out_bytes = align_up((size_t)vol(cext) * out_es);
    std::vector<size_t> inter;
    size_t scratch = 0;
    worst_layout(job.stages, p.core, job.n, inter, scratch);
    size_t set_bytes = in_bytes + n_out * out_bytes + scratch;
    for (size_t b : inter) set_bytes += b;

    DevBuf arena;
    arena.alloc(set_bytes * NB);
    struct Set {
        void *in, *out, *out2, *scratch;
        std::vector<void *> inter;
    };
    std::vector<Set> sets(NB);
    for (int b = 0; b < NB; ++b) {
        char *cur = static_cast<char *>(arena.p) + set_bytes * b;
        sets[b].in = cur;
        cur += in_bytes;
        sets[b].out = cur;
        cur += out_bytes;
        sets[b].out2 = n_out > 1 ? cur : nullptr;
        cur += (n_out - 1) * out_bytes;
        sets[b].inter.assign(job.stages.size(), nullptr);
        for (size_t k = 0; k < inter.size(); ++k) {
            sets[b].inter[k] = cur;
            cur += inter[k];
        }
        sets[b].scratch = scratch ? cur : nullptr;
    }

    // Pageable volumes go through pinned staging buffers.
    const bool stage_in = (min == Mem::Pageable), stage_out = (mout == Mem::Pageable);
    PinBuf pin_in, pin_out;
    if (stage_in) pin_in.alloc(in_bytes * NB);
    if (stage_out) pin_out.alloc(out_bytes * n_out * NB);

    StreamH s_h2d, s_comp, s_d2h;
    std::vector<EventH> ev_h2d(NB), ev_comp(NB), ev_d2h(NB);
    // With stats: timing events around each chunk's kernels on the compute
    // stream (their sum is the kernel time of the streamed run).
    std::vector<std::unique_ptr<EventH>> ev_k;
    if (stats) {
        ev_k.reserve((size_t)(2 * p.n_chunks));
        for (int64_t i = 0; i < 2 * p.n_chunks; ++i) ev_k.emplace_back(new EventH(true));
    }
    std::vector<int64_t> pending(NB, -1);  // chunk whose output awaits scatter

    int64_t bytes_h2d = 0, bytes_d2h = 0;
    void *host_in = const_cast<void *>(job.in);
    void *host_out[2] = {job.out, job.out2};

    auto finish_output = [&](int b) {
        const int64_t j = pending[b];
        if (j < 0) return;
        pending[b] = -1;
        if (!stage_out) return;
        int64_t d0[3], d1[3];
        chunk_box(p, j, d0, d1);
        check_hip(hipEventSynchronize(ev_d2h[b].e), "hipEventSynchronize");
        for (int o = 0; o < n_out; ++o)
            host_box_copy(false, host_out[o], out_es, job.n, d0, d1,
                          static_cast<char *>(pin_out.p) + (size_t)(b * n_out + o) * out_bytes);
    };

    for (int64_t i = 0; i < p.n_chunks; ++i) {
        const int b = (int)(i % NB);
        finish_output(b);
        chunk_box(p, i, c0, c1);
        expand(c0, c1, hh, job.n, lo, hi);
        for (int a = 0; a < 3; ++a) {
            iext[a] = hi[a] - lo[a];
            cext[a] = c1[a] - c0[a];
        }
        Set &S = sets[b];

        // H2D: the input buffer of set b is free once its last compute ended.
        if (i >= NB) check_hip(hipStreamWaitEvent(s_h2d.s, ev_comp[b].e, 0), "hipStreamWaitEvent");
        if (stage_in) {
            void *pin = static_cast<char *>(pin_in.p) + (size_t)b * in_bytes;
            if (i >= NB) check_hip(hipEventSynchronize(ev_h2d[b].e), "hipEventSynchronize");
            host_box_copy(true, host_in, in_es, job.n, lo, hi, pin);
            check_hip(hipMemcpyAsync(S.in, pin, (size_t)vol(iext) * in_es, hipMemcpyHostToDevice, s_h2d.s),
                      "hipMemcpyAsync");
        } else {
            Copy3D::run(true, host_in, in_es, job.n, lo, hi, S.in, s_h2d.s);
        }
        bytes_h2d += vol(iext) * (int64_t)in_es;
        check_hip(hipEventRecord(ev_h2d[b].e, s_h2d.s), "hipEventRecord");

        // Compute: needs the input, and the output buffer drained.
        check_hip(hipStreamWaitEvent(s_comp.s, ev_h2d[b].e, 0), "hipStreamWaitEvent");
        if (i >= NB) check_hip(hipStreamWaitEvent(s_comp.s, ev_d2h[b].e, 0), "hipStreamWaitEvent");
        const Region rin = dense_region(S.in, lo, hi);
        const Region rout = dense_region(S.out, c0, c1);
        Region rout2;
        if (n_out > 1) rout2 = dense_region(S.out2, c0, c1);
        if (stats) check_hip(hipEventRecord(ev_k[2 * i]->e, s_comp.s), "hipEventRecord");
        run_chunk_stages(job, rin, rout, n_out > 1 ? &rout2 : nullptr, c0, c1, S.inter.data(), S.scratch, scratch,
                         s_comp.s);
        if (stats) check_hip(hipEventRecord(ev_k[2 * i + 1]->e, s_comp.s), "hipEventRecord");
        check_hip(hipEventRecord(ev_comp[b].e, s_comp.s), "hipEventRecord");

        // D2H of the core.
        check_hip(hipStreamWaitEvent(s_d2h.s, ev_comp[b].e, 0), "hipStreamWaitEvent");
        for (int o = 0; o < n_out; ++o) {
            void *dsrc = o == 0 ? S.out : S.out2;
            if (stage_out) {
                void *pin = static_cast<char *>(pin_out.p) + (size_t)(b * n_out + o) * out_bytes;
                check_hip(hipMemcpyAsync(pin, dsrc, (size_t)vol(cext) * out_es, hipMemcpyDeviceToHost, s_d2h.s),
                          "hipMemcpyAsync");
            } else {
                Copy3D::run(false, host_out[o], out_es, job.n, c0, c1, dsrc, s_d2h.s);
            }
            bytes_d2h += vol(cext) * (int64_t)out_es;
        }
        check_hip(hipEventRecord(ev_d2h[b].e, s_d2h.s), "hipEventRecord");
        pending[b] = i;
    }
    for (int64_t i = std::max<int64_t>(0, p.n_chunks - NB); i < p.n_chunks; ++i) finish_output((int)(i % NB));
    check_hip(hipStreamSynchronize(s_h2d.s), "hipStreamSynchronize");
    check_hip(hipStreamSynchronize(s_comp.s), "hipStreamSynchronize");
    check_hip(hipStreamSynchronize(s_d2h.s), "hipStreamSynchronize");
    if (stats) {
        double kms = 0.0;
        for (int64_t i = 0; i < p.n_chunks; ++i) {
            float t = 0.f;
            check_hip(hipEventElapsedTime(&t, ev_k[2 * i]->e, ev_k[2 * i + 1]->e), "hipEventElapsedTime");
            kms += t;
        }
        stats->kernel_ms = kms;
        stats->n_chunks = p.n_chunks;
        stats->bytes_h2d = bytes_h2d;
        stats->bytes_d2h = bytes_d2h;
        stats->peak_device_bytes = (int64_t)(set_bytes * NB);
        stats->budget_bytes = (int64_t)budget;
    }
}

}  // namespace

// ------------------------------------------------------------ public pieces

size_t chunk_bytes(const ChunkCost &c, const int64_t core[3], const int64_t n[3])
{
    std::vector<size_t> inter;
    size_t scratch = 0;
    worst_layout(*c.stages, core, n, inter, scratch);
    size_t total = scratch;
    for (size_t b : inter) total += b;
    if (c.host) {
        int64_t big[3], cc[3];
        for (int a = 0; a < 3; ++a) {
            int64_t h = 0;
            for (const Stage &st : *c.stages) h += st.r[a];
            cc[a] = std::min(core[a], n[a]);
            big[a] = std::min(n[a], cc[a] + 2 * h);
        }
        total += align_up((size_t)vol(big) * c.in_es);
        total += (size_t)c.n_out * align_up((size_t)vol(cc) * c.out_es);
    }
    return total;
}

void plan_chunks(const int64_t n[3], const int32_t halo[3], const int64_t chunk[3], const ChunkCost &cost,
                 size_t budget, int max_buffers, harpia_plan &p)
{
    for (int a = 0; a < 3; ++a) {
        p.shape[a] = n[a];
        p.halo[a] = halo[a];
    }
    const bool auto_slab = chunk == nullptr || (chunk[0] == 0 && chunk[1] == 0 && chunk[2] == 0);
    int64_t core[3];
    int nb = 0;
    if (!auto_slab) {
        for (int a = 0; a < 3; ++a) {
            if (chunk[a] < 0) fail(HARPIA_ERR_ARG, "chunk extents must be >= 0");
            core[a] = chunk[a] == 0 ? n[a] : std::min(chunk[a], n[a]);
        }
        const size_t one = chunk_bytes(cost, core, n);
        for (nb = max_buffers; nb >= 1; --nb)
            if (one * (size_t)nb <= budget) break;
        if (nb < 1)
            fail(HARPIA_ERR_BUDGET, "chunk needs " + std::to_string(one) + " device bytes, budget is " +
                                        std::to_string(budget));
    } else {
        core[1] = n[1];
        core[2] = n[2];
        // Deepest slab that fits with nb buffer sets; prefer more sets.
        int64_t best = 0;
        for (nb = max_buffers; nb >= 1; --nb) {
            int64_t lo = 0, hi = n[0];
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) / 2;
                core[0] = mid;
                if (chunk_bytes(cost, core, n) * (size_t)nb <= budget)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            best = lo;
            if (best >= 1) break;
        }
        if (best < 1) {
            core[0] = 1;
            fail(HARPIA_ERR_BUDGET, "a 1-slice chunk with its halo needs " +
                                        std::to_string(chunk_bytes(cost, core, n)) + " device bytes, budget is " +
                                        std::to_string(budget));
        }
        // Streamed volumes: cap the slab so transfers overlap with compute
        // over several chunks (about 1 GiB of staged input per chunk).
        if (cost.host) {
            const int64_t plane = n[1] * n[2] * (int64_t)cost.in_es;
            const int64_t cap = std::max<int64_t>(1, ((int64_t)1 << 30) / std::max<int64_t>(1, plane));
            best = std::min(best, std::max<int64_t>(cap, 4 * (int64_t)halo[0] + 1));
            best = std::min(best, n[0]);
        }
        core[0] = best;
    }
    int64_t total = 1;
    for (int a = 0; a < 3; ++a) {
        p.core[a] = core[a];
        p.grid[a] = (n[a] + core[a] - 1) / core[a];
        total *= p.grid[a];
    }
    if (nb > total) nb = (int)total;  // no more buffer sets than chunks
    p.n_chunks = total;
    p.n_buffers = nb;
    p.device_bytes = chunk_bytes(cost, core, n) * (size_t)nb;
    p.budget_bytes = budget;
}

size_t resolve_budget(const harpia_exec *ex)
{
    // cap: the caller's, else the environment's default, else none
    size_t cap = ex ? ex->device_budget_bytes : 0;
    if (!cap) {
        const char *env_b = std::getenv("HARPIA_DEVICE_BUDGET");
        if (env_b && *env_b) cap = (size_t)std::strtoull(env_b, nullptr, 10);
    }
    double frac = HARPIA_DEFAULT_BUDGET_FRACTION;
    if (ex && ex->budget_fraction > 0) {
        frac = ex->budget_fraction;
    } else {
        const char *env_f = std::getenv("HARPIA_BUDGET_FRACTION");
        if (env_f && *env_f) frac = std::atof(env_f);
    }
    if (!(frac > 0.0 && frac <= 1.0)) fail(HARPIA_ERR_ARG, "budget fraction must be in (0, 1]");
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev < 1) {
        (void)hipGetLastError();
        // no device to query: a plan-only call keeps the cap as given
        if (cap) return cap;
        fail(HARPIA_ERR_ARG, "an explicit device budget is needed without a device");
    }
    size_t free_b = 0, total_b = 0;
    check_hip(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    const size_t limit = (size_t)((double)free_b * frac);
    return cap ? std::min(cap, limit) : limit;
}

bool is_device_pointer(const void *ptr) { return classify(ptr) == Mem::Device; }

void reset_alloc_counter() { t_alloc_count = 0; }

void run_job(const Job &job)
{
    const auto t0 = std::chrono::steady_clock::now();
    t_alloc_count = 0;
    harpia_stats *stats = job.ex ? job.ex->stats : nullptr;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    const Mem min = classify(job.in), mout = classify(job.out);
    const bool dev_in = min == Mem::Device, dev_out = mout == Mem::Device;
    if (job.out2 && (classify(job.out2) == Mem::Device) != dev_out)
        fail(HARPIA_ERR_ARG, "both outputs must live in the same memory");
    if (dev_in != dev_out) fail(HARPIA_ERR_ARG, "in and out must both be device pointers or both host pointers");
    if (dev_in)
        run_device(job, stats);
    else
        run_host(job, min, mout, stats);
    if (stats) stats->wall_ms = ms_since(t0);
}

}  // namespace harpia
