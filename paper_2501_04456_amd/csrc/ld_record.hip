// Trajectory recording (section 2.2: results can be recorded in a binary file
// for viewing and post-processing, with only every j-th frame recorded in a
// fine-time-step run).
//
// Every `every` steps of ld_step the positions (FP32 of the FP64 hi + lo, in
// original order) are gathered on the device into one of four staging
// buffers, copied asynchronously into pinned host memory, and written to
// the file by a writer thread in step order once the copy's event has
// completed, so the GPU keeps stepping while frames are written.  When all
// four slots are in flight the stepping thread waits for the oldest.
//
// File: "LDTRAJ01", int64 n, int32 n_types, int32 every, int32 type[n];
// then frames of int64 step, FP64 t, FP64 R(t), float32 x[n][3].
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "ld_host.h"

namespace ld {

using host::fail;

constexpr int kRecSlots = 4;

struct Recorder {
    FILE* f = nullptr;
    int every = 1;
    int n = 0;
    int64_t step = 0;                  // host mirror of the device clock
    double t = 0.0;
    float* dev[kRecSlots] = {};
    float* host[kRecSlots] = {};
    hipEvent_t ev[kRecSlots] = {};
    int64_t fstep[kRecSlots] = {};
    double ft[kRecSlots] = {}, fR[kRecSlots] = {};
    bool busy[kRecSlots] = {};
    std::deque<int> pending;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    bool failed = false;
    int64_t frames = 0;
    std::thread writer;
};

namespace {

__global__ __launch_bounds__(256) void k_rec_gather(const float4* __restrict__ pos,
                                                    const float4* __restrict__ lo,
                                                    const int* __restrict__ oid, int n,
                                                    float* __restrict__ out) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const float4 h = pos[s], l = lo[s];
    float* o = out + 3 * (size_t)oid[s];
    o[0] = (float)((double)h.x + (double)l.x);
    o[1] = (float)((double)h.y + (double)l.y);
    o[2] = (float)((double)h.z + (double)l.z);
}

void writer_loop(Recorder* r) {
    for (;;) {
        int slot;
        {
            std::unique_lock<std::mutex> lk(r->mu);
            r->cv.wait(lk, [&] { return r->stop || !r->pending.empty(); });
            if (r->pending.empty()) return;          // stop requested, nothing left
            slot = r->pending.front();
        }
        bool ok = hipEventSynchronize(r->ev[slot]) == hipSuccess;
        if (ok) {
            ok = std::fwrite(&r->fstep[slot], sizeof(int64_t), 1, r->f) == 1 &&
                 std::fwrite(&r->ft[slot], sizeof(double), 1, r->f) == 1 &&
                 std::fwrite(&r->fR[slot], sizeof(double), 1, r->f) == 1 &&
                 std::fwrite(r->host[slot], sizeof(float), 3 * (size_t)r->n, r->f) ==
                     3 * (size_t)r->n;
        }
        {
            std::lock_guard<std::mutex> lk(r->mu);
            r->pending.pop_front();
            r->busy[slot] = false;
            if (ok) ++r->frames;
            else r->failed = true;
        }
        r->cv.notify_all();
    }
}

void rec_release(Recorder* r) {
    if (r->writer.joinable()) {
        {
            std::lock_guard<std::mutex> lk(r->mu);
            r->stop = true;
        }
        r->cv.notify_all();
        r->writer.join();
    }
    for (int k = 0; k < kRecSlots; ++k) {
        if (r->dev[k]) (void)hipFree(r->dev[k]);
        if (r->host[k]) (void)hipHostFree(r->host[k]);
        if (r->ev[k]) (void)hipEventDestroy(r->ev[k]);
    }
    if (r->f) std::fclose(r->f);
    r->f = nullptr;
}

}  // namespace

void rec_free(ld_ctx* c) {
    if (!c->rec) return;
    rec_release(c->rec);
    delete c->rec;
    c->rec = nullptr;
}

// After one enqueued step of size dt: advance the host clock and, on a
// multiple of `every`, queue a frame.
ld_status rec_after_step(ld_ctx* c, double dt, hipStream_t s) {
    Recorder* r = c->rec;
    r->t = r->t + dt;                  // the device clock's own arithmetic
    r->step += 1;
    if (r->step % r->every != 0) return LD_OK;
    int slot = -1;
    {
        std::unique_lock<std::mutex> lk(r->mu);
        r->cv.wait(lk, [&] {
            for (int k = 0; k < kRecSlots; ++k)
                if (!r->busy[k]) return true;
            return false;
        });
        for (int k = 0; k < kRecSlots; ++k)
            if (!r->busy[k]) {
                slot = k;
                break;
            }
        r->busy[slot] = true;
        if (r->failed) return fail(LD_EHIP, "writing a trajectory frame failed");
    }
    const int n = r->n;
    hipLaunchKernelGGL(k_rec_gather, dim3((n + 255) / 256), dim3(256), 0, s, c->pos, c->lo, c->oid,
                       n, r->dev[slot]);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(r->host[slot], r->dev[slot], sizeof(float) * 3 * (size_t)n,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(r->ev[slot], s));
    r->fstep[slot] = r->step;
    r->ft[slot] = r->t;
    r->fR[slot] = radius_at(c->R, r->t);
    {
        std::lock_guard<std::mutex> lk(r->mu);
        r->pending.push_back(slot);
    }
    r->cv.notify_all();
    return LD_OK;
}

}  // namespace ld

using namespace ld;
using namespace ld::host;

extern "C" {

ld_status ld_record_open(ld_ctx* c, const char* path, int32_t every) {
    g_err.clear();
    if (!c || !path) return fail(LD_EINVAL, "ctx and path are required");
    if (every < 1) return fail(LD_EINVAL, "every must be >= 1");
    if (c->rec) return fail(LD_ESTATE, "a recording is open (ld_record_close first)");
    Recorder* r = new (std::nothrow) Recorder();
    if (!r) return fail(LD_ENOMEM, "host allocation failed");
    r->every = every;
    r->n = (int)c->n;
    DevState ds;
    hipError_t e = hipMemcpyAsync(&ds, c->st, sizeof ds, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete r;
        return fail(LD_EHIP, "reading the step clock: %s", hipGetErrorString(e));
    }
    r->step = ds.step;
    r->t = ds.t;
    bool ok = true;
    for (int k = 0; k < kRecSlots && ok; ++k)
        ok = hipMalloc(&r->dev[k], sizeof(float) * 3 * c->n) == hipSuccess &&
             hipHostMalloc(&r->host[k], sizeof(float) * 3 * c->n, hipHostMallocDefault) ==
                 hipSuccess &&
             hipEventCreateWithFlags(&r->ev[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        rec_release(r);
        delete r;
        return fail(LD_ENOMEM, "cannot allocate the frame buffers");
    }
    r->f = std::fopen(path, "wb");
    if (!r->f) {
        rec_release(r);
        delete r;
        return fail(LD_EINVAL, "cannot open %s for writing", path);
    }
    std::vector<int32_t> typ((size_t)c->n);
    std::vector<int32_t> oid((size_t)c->n), ts((size_t)c->n);
    e = hipMemcpyAsync(ts.data(), c->typ, sizeof(int32_t) * c->n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(oid.data(), c->oid, sizeof(int32_t) * c->n, hipMemcpyDeviceToHost,
                           c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        rec_release(r);
        delete r;
        return fail(LD_EHIP, "reading the types: %s", hipGetErrorString(e));
    }
    for (size_t s = 0; s < ts.size(); ++s) typ[(size_t)oid[s]] = ts[s];
    const char magic[8] = {'L', 'D', 'T', 'R', 'A', 'J', '0', '1'};
    const int64_t n64 = c->n;
    const int32_t nt = c->p.n_types;
    ok = std::fwrite(magic, 1, 8, r->f) == 8 && std::fwrite(&n64, 8, 1, r->f) == 1 &&
         std::fwrite(&nt, 4, 1, r->f) == 1 && std::fwrite(&every, 4, 1, r->f) == 1 &&
         std::fwrite(typ.data(), 4, typ.size(), r->f) == typ.size();
    if (!ok) {
        rec_release(r);
        delete r;
        return fail(LD_EINVAL, "cannot write the header of %s", path);
    }
    r->writer = std::thread(writer_loop, r);
    c->rec = r;
    c->graph_len = -1;                 // steps are enqueued one by one while recording
    return LD_OK;
}

ld_status ld_record_close(ld_ctx* c, int64_t* frames) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    if (!c->rec) return fail(LD_ESTATE, "no recording is open");
    Recorder* r = c->rec;
    if (r->writer.joinable()) {
        {
            std::lock_guard<std::mutex> lk(r->mu);
            r->stop = true;
        }
        r->cv.notify_all();
        r->writer.join();
    }
    const bool failed = r->failed;
    const int64_t nf = r->frames;
    const bool closed = std::fclose(r->f) == 0;
    r->f = nullptr;
    rec_free(c);
    if (frames) *frames = nf;
    if (failed || !closed) return fail(LD_EHIP, "writing the trajectory file failed");
    return LD_OK;
}

}  // extern "C"
