// Query server: continuous batching over resident graphs.
//
// Requests (graph, query) enter a FIFO queue.  Worker threads, each with its
// own HIP stream and workspace, take work whenever they are free: the head
// request together with every queued request on the same graph (up to a batch
// limit), so requests that arrive while others run join the next pass instead
// of waiting for a whole batch to drain.  A request is admitted only when the
// device memory it needs fits in the budget next to the requests in flight;
// otherwise it waits at the head of the queue.  Several workers run at once,
// so their kernels overlap on the device.  Latency is measured from submit to
// the moment the result is ready on the host.
//
// Memory counted against the budget: the estimates of the passes in flight (a
// single query's buffers, or the plan of a batch) plus the buffers each
// worker's workspace keeps between passes.  A worker that
// finds the head request does not fit gives its own workspace back; freed
// blocks stay in the library's cache, which is handed back to the driver when
// cache and counted memory together pass the budget.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

#include "folty_internal.h"

namespace folty {

namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

} // namespace

struct Server {
    struct Req {
        int64_t ticket;
        Graph *g;
        folty_query q;
        double t_submit;
        int64_t bytes;
    };
    struct Done {
        Result *r = nullptr;
        int code = FOLTY_OK;
        std::string err;
    };
    int device = 0;
    int64_t budget = 0, in_use = 0, peak_use = 0; // in_use: estimates of the requests in flight
    std::vector<int64_t> kept;                    // per worker: bytes its workspace keeps
    int64_t kept_total = 0;
    int active = 0, peak_active = 0;              // passes running at once
    int64_t held() const { return in_use + kept_total; }
    bool fits(int64_t b) const { return held() + b <= budget; }
    int max_batch = 16;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req> queue;
    std::unordered_map<int64_t, Done> done;
    std::unordered_map<int64_t, char> taken; // tickets whose result was handed out
    int64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0, rejected = 0, batches = 0, batched_requests = 0;
    bool stop = false;
    std::vector<std::thread> workers;

    std::atomic<int64_t> trimmed_bytes{0};
    void worker_main(int me);
    void trim_if_over();
    ~Server();
};

void Server::worker_main(int me) {
    if (hipSetDevice(device) != hipSuccess) return;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return;
    std::unique_ptr<Workspace> ws(new Workspace());
    auto set_kept = [&](int64_t b) { // caller holds mu
        kept_total += b - kept[me];
        kept[me] = b;
    };
    for (;;) {
        std::vector<Req> take;
        int64_t bytes = 0;
        bool give_back = false;
        {
            std::unique_lock<std::mutex> lk(mu);
            // wake to start the head request, or to give this worker's buffers back
            // when the head does not fit
            cv_work.wait(lk, [&] {
                return stop || (!queue.empty() && (fits(queue.front().bytes) || kept[me] > 0));
            });
            if (stop && queue.empty()) break;
            if (queue.empty()) continue;
            if (!fits(queue.front().bytes)) {
                give_back = kept[me] > 0;
                if (give_back) set_kept(0);
            } else {
                // the head, plus queued requests on the same graph while the plan
                // of them all still fits
                Req head = queue.front();
                queue.pop_front();
                take.push_back(head);
                bytes = head.bytes;
                std::vector<folty_query> qs(1, head.q);
                for (auto it = queue.begin(); it != queue.end() && (int)take.size() < max_batch;) {
                    if (it->g == head.g) {
                        qs.push_back(it->q);
                        const int64_t b = plan_footprint(head.g, qs.data(), (int)qs.size());
                        if (fits(b)) {
                            bytes = b;
                            take.push_back(*it);
                            it = queue.erase(it);
                            continue;
                        }
                        qs.pop_back();
                    }
                    ++it;
                }
                in_use += bytes;
                peak_use = std::max(peak_use, held());
                active++;
                peak_active = std::max(peak_active, active);
                if (take.size() > 1) {
                    batches++;
                    batched_requests += (int64_t)take.size();
                }
            }
        }
        if (give_back) {
            {
                StreamScope sc(s);
                ws.reset(new Workspace());
            }
            trim_if_over();
            cv_work.notify_all();
            continue;
        }
        if (take.empty()) continue;
        std::vector<Done> out(take.size());
        const double t_start = now_ms();
        try {
            StreamScope sc(s);
            if (take.size() == 1) {
                out[0].r = run_query_on(take[0].g, take[0].q, *ws, s);
            } else {
                std::vector<folty_query> qs(take.size());
                std::vector<int32_t> qg(take.size(), 0);
                for (size_t i = 0; i < take.size(); i++) qs[i] = take[i].q;
                Plan *P = plan_create(&take[0].g, 1, qs.data(), qg.data(), (int)qs.size(), true);
                std::vector<Result *> rs(take.size(), nullptr);
                try {
                    plan_run(P, rs.data());
                } catch (...) {
                    plan_free(P);
                    throw;
                }
                plan_free(P);
                for (size_t i = 0; i < take.size(); i++) out[i].r = rs[i];
            }
        } catch (const Error &e) {
            for (auto &d : out) {
                delete d.r;
                d.r = nullptr;
                d.code = e.code;
                d.err = e.what();
            }
        } catch (const std::exception &e) {
            for (auto &d : out) {
                delete d.r;
                d.r = nullptr;
                d.code = FOLTY_EDEVICE;
                d.err = e.what();
            }
        }
        const double t_end = now_ms();
        const int64_t ws_bytes = (int64_t)ws->device_bytes();
        {
            std::lock_guard<std::mutex> lk(mu);
            in_use -= bytes;
            active--;
            set_kept(ws_bytes);
            peak_use = std::max(peak_use, held());
            for (size_t i = 0; i < take.size(); i++) {
                if (out[i].r) {
                    out[i].r->stats.queue_ms = t_start - take[i].t_submit;
                    out[i].r->stats.latency_ms = t_end - take[i].t_submit;
                    out[i].r->stats.batch_size = (int64_t)take.size();
                }
                done[take[i].ticket] = std::move(out[i]);
                completed++;
            }
        }
        trim_if_over();
        cv_done.notify_all();
        cv_work.notify_all();
    }
    {
        StreamScope sc(s);
        ws.reset();
    }
    (void)hipStreamSynchronize(s);
    dev_forget_stream(s);
    (void)hipStreamDestroy(s);
}

// blocks the library keeps cached count too once they would push the device
// past the budget: then the largest go back to the driver until they fit
void Server::trim_if_over() {
    int64_t h;
    {
        std::lock_guard<std::mutex> lk(mu);
        h = held();
    }
    if (h + (int64_t)dev_cached() > budget) {
        (void)hipSetDevice(device);
        trimmed_bytes += (int64_t)dev_trim_to((size_t)std::max<int64_t>(0, budget - h));
    }
}

Server::~Server() {
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
    }
    cv_work.notify_all();
    for (auto &t : workers)
        if (t.joinable()) t.join();
    for (auto &kv : done) delete kv.second.r;
}

Server *server_create(const folty_server_opts *o) {
    folty_server_opts opts{};
    if (o) opts = *o;
    if (opts.workers <= 0) opts.workers = 4;
    if (opts.workers > 64) fail(FOLTY_EINVAL, "at most 64 workers");
    if (opts.max_batch <= 0) opts.max_batch = 16;
    std::unique_ptr<Server> S(new Server());
    FOLTY_HIP(hipGetDevice(&S->device));
    int64_t budget = opts.hbm_budget_bytes;
    if (budget <= 0) {
        size_t free_b = 0, total_b = 0;
        FOLTY_HIP(hipMemGetInfo(&free_b, &total_b));
        budget = (int64_t)(free_b * 0.8);
    }
    S->budget = budget;
    S->max_batch = opts.max_batch;
    S->kept.assign(opts.workers, 0);
    for (int i = 0; i < opts.workers; i++) S->workers.emplace_back([s = S.get(), i] { s->worker_main(i); });
    return S.release();
}

int64_t server_submit(Server *S, Graph *g, const folty_query &q) {
    check_query(g, q);
    ensure_triangles(g); // the footprint bound needs the triangle count
    const int64_t bytes = query_footprint(g, q);
    std::lock_guard<std::mutex> lk(S->mu);
    if (bytes > S->budget) {
        S->rejected++;
        fail(FOLTY_ENOMEM, "query needs %lld bytes of device memory, budget is %lld", (long long)bytes,
             (long long)S->budget);
    }
    Server::Req r{S->next_ticket++, g, q, now_ms(), bytes};
    S->queue.push_back(r);
    S->submitted++;
    S->cv_work.notify_one();
    return r.ticket;
}

// FOLTY_EBUSY while the request is not done (wait = false)
Result *server_take(Server *S, int64_t ticket, bool wait) {
    std::unique_lock<std::mutex> lk(S->mu);
    if (ticket <= 0 || ticket >= S->next_ticket) fail(FOLTY_EINVAL, "unknown ticket %lld", (long long)ticket);
    if (S->taken.count(ticket)) fail(FOLTY_EINVAL, "ticket %lld was already taken", (long long)ticket);
    auto ready = [&] { return S->done.count(ticket) > 0; };
    if (!ready()) {
        if (!wait) fail(FOLTY_EBUSY, "not done");
        S->cv_done.wait(lk, ready);
    }
    Server::Done d = std::move(S->done[ticket]);
    S->done.erase(ticket);
    S->taken[ticket] = 1;
    if (!d.r) fail(d.code, "%s", d.err.c_str());
    return d.r;
}

void server_info(Server *S, folty_server_info *info) {
    std::lock_guard<std::mutex> lk(S->mu);
    info->submitted = S->submitted;
    info->completed = S->completed;
    info->rejected = S->rejected;
    info->queued = (int64_t)S->queue.size();
    info->batches = S->batches;
    info->batched_requests = S->batched_requests;
    info->budget_bytes = S->budget;
    info->in_use_bytes = S->held();
    info->peak_in_use_bytes = S->peak_use;
    info->kept_bytes = S->kept_total;
    info->peak_concurrent_passes = S->peak_active;
    info->trimmed_bytes = S->trimmed_bytes.load();
}

void server_destroy(Server *S) { delete S; }

} // namespace folty
