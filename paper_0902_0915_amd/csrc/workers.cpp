// Per-instance plan work spread over host threads. Building a plan of many small instances is
// bound by launch latency and host-device round trips (tens of launches and a few waits per
// instance), not by the device: several host threads, each issuing to a stream of its own,
// overlap those round trips and keep the device busy.
#include "internal.h"

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

namespace mwg {

namespace {
constexpr int kPlanThreads = 8;
}

Status parallel_instances(int device, int n, hipStream_t after, const std::function<Status(int, hipStream_t)> &job,
                          size_t tmp_first_block) {
    if (n <= 0) return Status::Ok();
    const int nt = std::min(kPlanThreads, n);
    hipEvent_t ready = nullptr;
    MWG_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    if (hipEventRecord(ready, after) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(ready);
        return make_error(MW_ERR_HIP, "hipEventRecord failed");
    }
    std::vector<Status> result((size_t)nt);
    std::atomic<int> next{0};
    std::atomic<bool> failed{false};
    auto worker = [&](int w) {
        Status &out = result[(size_t)w];
        try {
            hipStream_t s = nullptr;
            if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
                (void)hipGetLastError();
                out = make_error(MW_ERR_HIP, "worker stream set-up failed");
                failed = true;
                return;
            }
            if (hipStreamWaitEvent(s, ready, 0) != hipSuccess) {  // device inputs written on `after`
                (void)hipGetLastError();
                out = make_error(MW_ERR_HIP, "hipStreamWaitEvent failed");
                failed = true;
            } else {
                TmpScope scope(s, tmp_first_block);  // this thread's temporaries; waits for s when it ends
                for (int i = next++; i < n && !failed; i = next++) {
                    Status r = job(i, s);
                    if (!r.ok()) {
                        out = r;
                        failed = true;
                        break;
                    }
                }
            }
            if (hipStreamSynchronize(s) != hipSuccess && out.ok()) {
                (void)hipGetLastError();
                out = make_error(MW_ERR_HIP, "hipStreamSynchronize failed in a plan worker");
                failed = true;
            }
            (void)hipStreamDestroy(s);
        } catch (const std::bad_alloc &) {
            out = make_error(MW_ERR_ALLOC, "host allocation failed in a plan worker");
            failed = true;
        } catch (...) {
            out = make_error(MW_ERR_HIP, "unexpected exception in a plan worker");
            failed = true;
        }
    };
    std::vector<std::thread> threads;
    threads.reserve((size_t)nt);
    for (int w = 0; w < nt; w++) {
        try {
            threads.emplace_back(worker, w);
        } catch (...) {
            break;  // the threads that started take all the work
        }
    }
    if (threads.empty()) worker(0);
    for (std::thread &t : threads) t.join();
    (void)hipEventDestroy(ready);
    for (const Status &r : result)
        if (!r.ok()) return r;
    return Status::Ok();
}

} // namespace mwg
