// dsd_server_*: continuous batching of densest-subgraph queries.
//
// A server owns WORKERS worker threads, each with a non-blocking HIP stream
// of its own (default priority).  A worker that is free takes the next work
// from the queue at once: the oldest queued request, and with it, when that
// request is on a small graph, every other queued small request with the same
// op and h on a distinct graph whose device footprint still fits the budget
// (at most MAX_GROUP); a request on a large graph runs alone.  The group runs
// through the batch path on the worker's stream: every handle of the group is
// switched to that stream for the run and switched back afterwards.  So
// requests that arrive while others are on the GPU start as soon as a worker
// and enough of the budget are free, and the groups of different workers
// overlap on the device.  At most WORKERS - 1 workers hold large requests at
// a time, so small requests never wait behind large ones alone.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <deque>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "handle.hpp"

namespace {

constexpr size_t BYTES_PER_VERTEX = 160;
constexpr size_t BYTES_PER_EDGE = 192;
constexpr size_t MAX_GROUP = 4096;
constexpr int64_t LARGE_EDGES = (int64_t)1 << 20;   // a request on a larger graph runs alone
constexpr int WORKERS_DEFAULT = 4;

enum class St { QUEUED, RUNNING, DONE, CANCELED };

struct Req {
    uint64_t ticket;
    dsd_graph g;
    int h, op, out_mem;
    void *out;
    size_t foot;
};

int workers_wanted() {
    const char *e = std::getenv("DSD_SERVER_WORKERS");
    const int w = e ? std::atoi(e) : WORKERS_DEFAULT;
    return std::max(2, std::min(16, w));
}

}  // namespace

struct dsd_server_s {
    size_t budget = 0;
    int max_slots = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req> queue;
    std::unordered_map<uint64_t, St> state;
    std::unordered_map<uint64_t, dsd_result> done;
    uint64_t next_ticket = 1;
    int in_flight = 0;     // queued + running
    size_t running = 0;    // footprints of the groups being run
    int large_running = 0; // workers holding a large request
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;

    static bool large(const Req &r) { return r.g->g.m >= LARGE_EDGES; }

    // the next group a free worker can run (mu held); empty if none
    std::vector<Req> take() {
        std::vector<Req> group;
        const int nw = (int)workers.size();
        size_t used = 0;
        std::set<dsd_graph> seen;
        int op = -1, h = -1;
        for (auto it = queue.begin(); it != queue.end() && group.size() < MAX_GROUP;) {
            const bool lg = large(*it);
            if (group.empty()) {
                // the oldest request that may start now leads the group
                const bool fits = running + it->foot <= budget || running == 0;
                if (!fits || (lg && large_running >= nw - 1)) {
                    ++it;
                    continue;
                }
                op = it->op;
                h = it->h;
                used = it->foot;
                seen.insert(it->g);
                state[it->ticket] = St::RUNNING;
                group.push_back(*it);
                it = queue.erase(it);
                if (lg) break;                      // a large graph runs alone
                continue;
            }
            if (!lg && it->op == op && it->h == h && !seen.count(it->g) && running + used + it->foot <= budget) {
                used += it->foot;
                seen.insert(it->g);
                state[it->ticket] = St::RUNNING;
                group.push_back(*it);
                it = queue.erase(it);
            } else {
                ++it;
            }
        }
        return group;
    }

    void run(int w) {
        hipStream_t ws = streams[w];
        while (true) {
            std::vector<Req> group;
            size_t foot = 0;
            bool lg = false;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    if (stop && queue.empty()) return true;
                    group = take();
                    return !group.empty();
                });
                if (group.empty()) return;          // stopping, nothing queued
                for (const Req &r : group) foot += r.foot;
                lg = large(group[0]);
                running += foot;
                large_running += lg ? 1 : 0;
            }
            const int32_t cnt = (int32_t)group.size();
            std::vector<dsd_result> res(cnt);
            // the group runs on this worker's stream
            std::vector<hipStream_t> own(cnt);
            for (int32_t i = 0; i < cnt; i++) {
                own[i] = group[i].g->stream;
                (void)hipStreamSynchronize(own[i]);
                group[i].g->stream = ws;
            }
            // requests with host and with device outputs go in two calls
            for (int pass = 0; pass < 2; pass++) {
                const int mem = pass == 0 ? DSD_MEM_HOST : DSD_MEM_DEVICE;
                std::vector<int32_t> sel;
                for (int32_t i = 0; i < cnt; i++)
                    if ((group[i].out ? group[i].out_mem : DSD_MEM_HOST) == mem) sel.push_back(i);
                if (sel.empty()) continue;
                std::vector<dsd_graph> g2;
                std::vector<int> h2;
                std::vector<void *> o2;
                std::vector<dsd_result> r2(sel.size());
                for (int32_t i : sel) {
                    g2.push_back(group[i].g);
                    h2.push_back(group[i].h);
                    o2.push_back(group[i].out);
                }
                const dsd_status st = dsd_batch_run((int32_t)sel.size(), g2.data(), h2.data(), group[0].op, mem,
                                                    o2.data(), r2.data());
                for (size_t j = 0; j < sel.size(); j++) {
                    res[sel[j]] = r2[j];
                    if (st == DSD_EINVAL) res[sel[j]].status = DSD_EINVAL;
                }
            }
            (void)hipStreamSynchronize(ws);
            for (int32_t i = 0; i < cnt; i++) group[i].g->stream = own[i];
            {
                std::lock_guard<std::mutex> lk(mu);
                running -= foot;
                large_running -= lg ? 1 : 0;
                for (int32_t i = 0; i < cnt; i++) {
                    state[group[i].ticket] = St::DONE;
                    done[group[i].ticket] = res[i];
                    in_flight--;
                }
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

using namespace dsd;

extern "C" {

dsd_status dsd_server_create(size_t hbm_budget_bytes, int max_slots, dsd_server *out) {
    if (!out) return fail(DSD_EINVAL, "NULL output handle");
    *out = nullptr;
    if (hbm_budget_bytes == 0 || max_slots <= 0) return fail(DSD_EINVAL, "budget and slots must be positive");
    DSD_TRY({
        check_device();
        std::unique_ptr<dsd_server_s> s(new dsd_server_s());
        s->budget = hbm_budget_bytes;
        s->max_slots = max_slots;
        const int nw = workers_wanted();
        for (int w = 0; w < nw; w++) {
            hipStream_t st = nullptr;
            const hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (e != hipSuccess) {
                for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
                throw Error(DSD_EDEVICE, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
            }
            s->streams.push_back(st);
        }
        dsd_server_s *p = s.release();
        for (int w = 0; w < nw; w++) p->workers.emplace_back([p, w] { p->run(w); });
        *out = p;
        return DSD_OK;
    })
}

dsd_status dsd_server_submit(dsd_server s, dsd_graph g, int h, int op, int out_mem, void *out, uint64_t *ticket) {
    if (!s || !g || !ticket) return fail(DSD_EINVAL, "NULL argument");
    if (h < 2 || h > 6) return fail(DSD_EINVAL, "h must be in [2, 6]");
    if (op < DSD_OP_DEGREES || op > DSD_OP_PEEL) return fail(DSD_EINVAL, "unknown operation");
    if (out && out_mem != DSD_MEM_HOST && out_mem != DSD_MEM_DEVICE) return fail(DSD_EINVAL, "bad memory flag");
    const size_t foot = BYTES_PER_VERTEX * (size_t)g->g.n + BYTES_PER_EDGE * (size_t)g->g.m;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(DSD_EINVAL, "server is shutting down");
    if (foot > s->budget) return fail(DSD_ENOMEM, "request footprint exceeds the server's device-memory budget");
    if (s->in_flight >= s->max_slots) return fail(DSD_EBUSY, "no free request slot");
    const uint64_t t = s->next_ticket++;
    s->queue.push_back(Req{t, g, h, op, out_mem, out, foot});
    s->state[t] = St::QUEUED;
    s->in_flight++;
    *ticket = t;
    s->cv_work.notify_one();
    return DSD_OK;
}

dsd_status dsd_server_wait(dsd_server s, uint64_t ticket, int64_t timeout_us, dsd_result *out) {
    if (!s) return fail(DSD_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] {
        auto it = s->state.find(ticket);
        return it == s->state.end() || it->second == St::DONE || it->second == St::CANCELED;
    };
    if (timeout_us < 0) s->cv_done.wait(lk, ready);
    else s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    auto it = s->state.find(ticket);
    if (it == s->state.end()) return fail(DSD_EINVAL, "unknown ticket");
    if (it->second == St::CANCELED) {
        s->state.erase(it);
        return DSD_ECANCELED;
    }
    if (it->second != St::DONE) return DSD_ETIMEDOUT;
    if (out) *out = s->done[ticket];
    s->done.erase(ticket);
    s->state.erase(it);
    return DSD_OK;
}

dsd_status dsd_server_cancel(dsd_server s, uint64_t ticket) {
    if (!s) return fail(DSD_EINVAL, "NULL server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->state.find(ticket);
        if (it == s->state.end()) return fail(DSD_EINVAL, "unknown ticket");
        if (it->second != St::QUEUED) return DSD_EBUSY;
        for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
            if (q->ticket == ticket) {
                s->queue.erase(q);
                break;
            }
        it->second = St::CANCELED;
        s->in_flight--;
    }
    s->cv_done.notify_all();
    return DSD_OK;
}

dsd_status dsd_server_destroy(dsd_server s) {
    if (!s) return DSD_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (const Req &r : s->queue) s->state[r.ticket] = St::CANCELED;
        s->in_flight -= (int)s->queue.size();
        s->queue.clear();
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    for (std::thread &w : s->workers)
        if (w.joinable()) w.join();
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return DSD_OK;
}

}  // extern "C"
