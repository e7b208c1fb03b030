// dsd_server_*: a request queue served through the batch path by two worker
// threads, one for graphs below LARGE_EDGES edges and one for larger ones.
// A worker takes, in arrival order, queued requests of its class with the
// first one's op whose graphs are distinct and whose estimated device
// footprints fit what the budget leaves, runs them as one batch (a large
// graph alone) and completes their tickets.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
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
constexpr int64_t LARGE_EDGES = (int64_t)1 << 20;   // requests on larger graphs go to the second worker

enum class St { QUEUED, RUNNING, DONE, CANCELED };

struct Req {
    uint64_t ticket;
    dsd_graph g;
    int h, op, out_mem;
    void *out;
    size_t foot;
};

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
    bool stop = false;
    std::thread workers[2];

    static bool large(const Req &r) { return r.g->g.m >= LARGE_EDGES; }

    bool has_class(bool lg) const {
        for (const Req &r : queue)
            if (large(r) == lg) return true;
        return false;
    }

    // the next group of class lg that fits the budget left (mu held); empty if none
    std::vector<Req> take(bool lg) {
        std::vector<Req> group;
        int op = -1;
        size_t used = 0;
        std::set<dsd_graph> seen;
        for (auto it = queue.begin(); it != queue.end() && group.size() < MAX_GROUP;) {
            if (large(*it) != lg) {
                ++it;
                continue;
            }
            if (op < 0) op = it->op;
            const bool fits = running + used + it->foot <= budget || (running == 0 && group.empty());
            if (it->op == op && !seen.count(it->g) && fits) {
                used += it->foot;
                seen.insert(it->g);
                state[it->ticket] = St::RUNNING;
                group.push_back(*it);
                it = queue.erase(it);
            } else {
                ++it;
            }
            if (lg && !group.empty()) break;    // a large graph runs alone
        }
        return group;
    }

    void run(bool lg) {
        while (true) {
            std::vector<Req> group;
            size_t foot = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    if (stop && !has_class(lg)) return true;
                    group = take(lg);
                    return !group.empty();
                });
                if (group.empty()) return;          // stopping, nothing of this class queued
                for (const Req &r : group) foot += r.foot;
                running += foot;
            }
            const int32_t cnt = (int32_t)group.size();
            std::vector<dsd_result> res(cnt);
            // one op per group; requests with host and with device outputs go in two calls
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
                dsd_status st = dsd_batch_run((int32_t)sel.size(), g2.data(), h2.data(), group[0].op, mem, o2.data(),
                                              r2.data());
                for (size_t j = 0; j < sel.size(); j++) {
                    res[sel[j]] = r2[j];
                    if (st == DSD_EINVAL) res[sel[j]].status = DSD_EINVAL;
                }
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                running -= foot;
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
        dsd_server_s *s = new dsd_server_s();
        s->budget = hbm_budget_bytes;
        s->max_slots = max_slots;
        s->workers[0] = std::thread([s] { s->run(false); });
        s->workers[1] = std::thread([s] { s->run(true); });
        *out = s;
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
    s->cv_work.notify_all();    // two workers: wake the one of this request's class
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
    delete s;
    return DSD_OK;
}

}  // extern "C"
