// host_stream.hip -- fills from events in host memory, pipelined.
//
// The paper's CUDA histogram (arXiv:2401.13310 Sec. 3.2) copies every bulk of
// events from the host to the device before its fill kernel, and its time is
// dominated by those transfers and the per-bulk API overhead (Sec. 4.4, Sec. 6,
// where overlapping them is named as future work).  Sec. 3.3 records the
// hazard of that design: a host buffer refilled with the next bulk while the
// previous copy still reads it.
//
// hist_fill_host streams the events in chunks through two slots.  Each slot
// owns a device buffer and, for pageable input, a page-locked host staging
// buffer.  Chunk i (slot i mod 2):
//   1. host threads copy the chunk's columns into the slot's staging buffer,
//      after waiting for the slot's previous host->device copy (so the staging
//      buffer is never rewritten while the DMA engine reads it: the Sec. 3.3
//      race);
//   2. the copy stream waits until the fill that last read the slot's device
//      buffer has run, then copies the chunk host->device;
//   3. the fill stream waits for that copy and runs the ordinary fill.
// The copy of chunk i+1 and the host staging of chunk i+2 thus overlap the
// fill of chunk i.  Page-locked input (HIST_HOST_PINNED) skips step 1.
#include "../../include/hist.h"
#include "kernels.h"
#include "plan.h"

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace hg {

// A small process-wide pool of host threads for the staging copies: a single
// thread copies pageable memory at well under the host->device link rate.
class CopyPool {
public:
    static CopyPool &get()
    {
        static CopyPool pool;
        return pool;
    }

    // Copies `bytes` from src to dst, split over the pool's threads; returns
    // when every part is done.
    void copy(void *dst, const void *src, size_t bytes)
    {
        const size_t kMinPart = (size_t)1 << 20;
        const int parts = (int)std::min<size_t>(workers_.size() + 1, std::max<size_t>(1, bytes / kMinPart));
        if (parts <= 1) {
            std::memcpy(dst, src, bytes);
            return;
        }
        const size_t per = (bytes + parts - 1) / parts;
        std::unique_lock<std::mutex> lock(mu_);
        for (int p = 1; p < parts; ++p) {
            const size_t o = (size_t)p * per;
            const size_t len = o < bytes ? std::min(per, bytes - o) : 0;
            jobs_.push_back([=] {
                if (len)
                    std::memcpy(static_cast<char *>(dst) + o, static_cast<const char *>(src) + o, len);
            });
        }
        pending_ += parts - 1;
        lock.unlock();
        cv_.notify_all();
        std::memcpy(dst, src, std::min(per, bytes));
        lock.lock();
        done_cv_.wait(lock, [&] { return pending_ == 0; });
    }

private:
    CopyPool()
    {
        const unsigned hw = std::thread::hardware_concurrency();
        const int n = (int)std::max(1u, std::min(hw ? hw : 1u, 8u)) - 1;
        for (int i = 0; i < n; ++i)
            workers_.emplace_back([this] { run(); });
    }
    ~CopyPool()
    {
        {
            std::lock_guard<std::mutex> lock(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : workers_)
            t.join();
    }
    void run()
    {
        std::unique_lock<std::mutex> lock(mu_);
        for (;;) {
            cv_.wait(lock, [&] { return stop_ || !jobs_.empty(); });
            if (stop_ && jobs_.empty())
                return;
            auto job = std::move(jobs_.back());
            jobs_.pop_back();
            lock.unlock();
            job();
            lock.lock();
            if (--pending_ == 0)
                done_cv_.notify_all();
        }
    }

    std::vector<std::thread> workers_;
    std::vector<std::function<void()>> jobs_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    int pending_ = 0;
    bool stop_ = false;
};

struct HostSlot {
    void *host = nullptr;     // page-locked staging (pageable input only)
    void *dev = nullptr;      // device columns of one chunk
    hipEvent_t copied = nullptr;    // host->device copy of the slot done
    hipEvent_t consumed = nullptr;  // the fill reading the slot's device buffer done
    bool used = false;
};

struct HostStreamer {
    hipStream_t copy = nullptr;
    size_t slot_bytes = 0;     // bytes of one slot's buffers
    bool staging = false;      // host staging buffers allocated
    HostSlot slot[2];
};

void host_streamer_destroy(HostStreamer *hs)
{
    if (!hs)
        return;
    if (hs->copy) {
        (void)hipStreamSynchronize(hs->copy);
        (void)hipStreamDestroy(hs->copy);
    }
    for (HostSlot &s : hs->slot) {
        if (s.consumed)
            (void)hipEventSynchronize(s.consumed);
        if (s.host)
            (void)hipHostFree(s.host);
        if (s.dev)
            (void)hipFree(s.dev);
        if (s.copied)
            (void)hipEventDestroy(s.copied);
        if (s.consumed)
            (void)hipEventDestroy(s.consumed);
    }
    delete hs;
    (void)hipGetLastError();
}

// Buffers for chunks of `bytes` per slot (and staging when asked); keeps
// larger buffers.  Waits for work still using buffers it replaces.
static hist_status streamer_ready(hist_s *h, size_t bytes, bool staging)
{
    if (!h->host) {
        h->host = new (std::nothrow) HostStreamer();
        if (!h->host)
            return set_error(HIST_ENOMEM, "hist_fill_host: host allocation");
        if (hipStreamCreateWithFlags(&h->host->copy, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            h->host->copy = nullptr;
            return set_error(HIST_EDEVICE, "hist_fill_host: copy stream");
        }
        for (HostSlot &s : h->host->slot) {
            if (hipEventCreateWithFlags(&s.copied, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&s.consumed, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                return set_error(HIST_EDEVICE, "hist_fill_host: events");
            }
        }
    }
    HostStreamer &hs = *h->host;
    const bool grow = bytes > hs.slot_bytes;
    if (!grow && (!staging || hs.staging))
        return HIST_OK;
    const size_t nb = std::max(bytes, hs.slot_bytes);
    for (HostSlot &s : hs.slot) {
        if (s.used) {
            (void)hipEventSynchronize(s.copied);
            (void)hipEventSynchronize(s.consumed);
        }
        if (grow) {
            if (s.dev)
                (void)hipFree(s.dev);
            s.dev = nullptr;
            if (hipMalloc(&s.dev, nb) != hipSuccess) {
                (void)hipGetLastError();
                hs.slot_bytes = 0;
                return set_error(HIST_ENOMEM, "hist_fill_host: device chunk buffer of %zu bytes", nb);
            }
        }
        if (staging && (grow || !s.host)) {
            if (s.host)
                (void)hipHostFree(s.host);
            s.host = nullptr;
            if (hipHostMalloc(&s.host, nb, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                hs.staging = false;
                return set_error(HIST_ENOMEM, "hist_fill_host: page-locked staging of %zu bytes", nb);
            }
        }
        s.used = false;
    }
    hs.slot_bytes = nb;
    if (staging)
        hs.staging = true;
    return HIST_OK;
}

}  // namespace hg

using namespace hg;

extern "C" hist_status hist_fill_host(hist_t *h, const void *const *coords, const void *weights,
                                      int64_t n, hist_dtype dtype, int64_t chunk, uint32_t flags,
                                      void *stream)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_fill_host: NULL handle");
    if (dtype != HIST_F64 && dtype != HIST_F32)
        return set_error(HIST_EINVAL, "hist_fill_host: unknown dtype %d", (int)dtype);
    if (flags & ~(uint32_t)HIST_HOST_PINNED)
        return set_error(HIST_EINVAL, "hist_fill_host: unknown flags 0x%x", flags);
    if (n < 0 || chunk < 0)
        return set_error(HIST_EINVAL, "hist_fill_host: need n >= 0 and chunk >= 0");
    if (n == 0)
        return HIST_OK;
    if (!coords)
        return set_error(HIST_EINVAL, "hist_fill_host: coords is NULL");
    for (int a = 0; a < h->dims; ++a)
        if (!coords[a])
            return set_error(HIST_EINVAL, "hist_fill_host: coordinate %d is NULL", a);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess)
        (void)hipGetLastError();
    if (cs != hipStreamCaptureStatusNone)
        return set_error(HIST_ECAPTURE, "hist_fill_host: stream is capturing");

    const bool pinned = (flags & HIST_HOST_PINNED) != 0;
    const bool weighted = weights != nullptr;
    const size_t esz = dtype == HIST_F32 ? 4 : 8;
    const int ncol = h->dims + (weighted ? 1 : 0);
    if (chunk == 0)
        chunk = kHostChunkDefault;
    if (chunk > n)
        chunk = n;
    // scratch of the plan for a full chunk (a shorter last chunk needs less)
    hist_status st = reserve_scratch(h, chunk, dtype, weighted, s);
    if (st != HIST_OK)
        return st;
    const size_t col_bytes = (size_t)chunk * esz;
    st = streamer_ready(h, col_bytes * ncol, !pinned);
    if (st != HIST_OK)
        return st;
    HostStreamer &hs = *h->host;
    const Plan p_full = make_plan(h, chunk, dtype, weighted);
    const void *src[kMaxDims + 1];
    for (int a = 0; a < h->dims; ++a)
        src[a] = coords[a];
    if (weighted)
        src[h->dims] = weights;

    (void)hipGetLastError();
    int64_t i = 0;
    for (int64_t off = 0; off < n; off += chunk, ++i) {
        const int64_t m = std::min<int64_t>(chunk, n - off);
        HostSlot &sl = hs.slot[i & 1];
        const size_t mb = (size_t)m * esz;
        // (1) the staging buffer is free once its previous copy has run
        if (!pinned) {
            if (sl.used && hipEventSynchronize(sl.copied) != hipSuccess)
                return set_error(HIST_EDEVICE, "hist_fill_host: waiting for a copy");
            for (int c = 0; c < ncol; ++c)
                CopyPool::get().copy(static_cast<char *>(sl.host) + c * col_bytes,
                                     static_cast<const char *>(src[c]) + off * esz, mb);
        }
        // (2) the device buffer is free once the fill that read it has run
        if (sl.used && hipStreamWaitEvent(hs.copy, sl.consumed, 0) != hipSuccess)
            return set_error(HIST_EDEVICE, "hist_fill_host: stream wait");
        for (int c = 0; c < ncol; ++c) {
            const void *from = pinned ? static_cast<const char *>(src[c]) + off * esz
                                      : static_cast<const char *>(sl.host) + c * col_bytes;
            if (hipMemcpyAsync(static_cast<char *>(sl.dev) + c * col_bytes, from, mb,
                               hipMemcpyHostToDevice, hs.copy) != hipSuccess) {
                (void)hipGetLastError();
                return set_error(HIST_EDEVICE, "hist_fill_host: host->device copy");
            }
        }
        if (hipEventRecord(sl.copied, hs.copy) != hipSuccess ||
            hipStreamWaitEvent(s, sl.copied, 0) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(HIST_EDEVICE, "hist_fill_host: copy event");
        }
        sl.used = true;
        // (3) the ordinary fill of the chunk on the caller's stream
        const void *dcols[kMaxDims];
        for (int a = 0; a < h->dims; ++a)
            dcols[a] = static_cast<const char *>(sl.dev) + a * col_bytes;
        const void *dw = weighted ? static_cast<const char *>(sl.dev) + h->dims * col_bytes : nullptr;
        const Plan p = m == chunk ? p_full : make_plan(h, m, dtype, weighted);
        st = run_plan(h, p, dcols, dw, m, dtype, s);
        if (st != HIST_OK)
            return st;
        if (hipEventRecord(sl.consumed, s) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(HIST_EDEVICE, "hist_fill_host: fill event");
        }
    }
    // page-locked input is read by the copy engine: the caller may reuse it
    // only once the last copies are done
    if (pinned && hipStreamSynchronize(hs.copy) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(HIST_EDEVICE, "hist_fill_host: copy synchronize");
    }
    return HIST_OK;
}
