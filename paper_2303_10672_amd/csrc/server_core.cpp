// Scheduling core of the request server (see server_core.h).  Plain C++17: no HIP.
#include "server_core.h"

#include <algorithm>
#include <cinttypes>

namespace pvi {
namespace srv {

Core::Core(const Config& cfg) : cfg_(cfg), t0_(clk::now()) {
    if (cfg_.recheck_us < 1) cfg_.recheck_us = 1;
    if (cfg_.log_path && cfg_.log_path[0]) log_ = std::fopen(cfg_.log_path, "a");
}

Core::~Core() {
    shutdown(0);
    if (log_) std::fclose(log_);
}

double Core::ms_since_start(clk::time_point t) const {
    return std::chrono::duration<double, std::milli>(t - t0_).count();
}

void Core::log_event(const char* what, const Job* j) {
    if (!log_) return;
    std::fprintf(log_, "%.3f %s ticket=%" PRIu64 " class=%s worker=%d bytes=%" PRId64
                       " status=%d\n",
                 ms_since_start(clk::now()), what, j->ticket, j->small ? "small" : "large",
                 j->worker, j->bytes, j->status);
    std::fflush(log_);
}

bool Core::submit(std::vector<std::unique_ptr<Job>>& jobs, uint64_t* tickets) {
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (stop_) return false;
        const auto now = clk::now();
        for (size_t i = 0; i < jobs.size(); ++i) {
            Job* j = jobs[i].get();
            j->ticket = next_ticket_++;
            j->state = kQueued;
            j->t_submit = now;
            tickets[i] = j->ticket;
            (j->small ? small_q_ : large_q_).push_back(j);
            log_event("submit", j);
            jobs_[j->ticket] = std::move(jobs[i]);
        }
    }
    jobs.clear();
    cv_work_.notify_all();
    return true;
}

int Core::wait(uint64_t ticket, int64_t timeout_us, Job** out) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return -1;
    Job* j = it->second.get();
    auto ready = [&] { return j->state == kDone; };
    if (timeout_us < 0)
        cv_done_.wait(lk, ready);
    else if (!cv_done_.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
        return 0;
    if (out) *out = j;
    return 1;
}

int Core::poll(uint64_t ticket, Job** out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return -1;
    if (out) *out = it->second.get();
    return it->second->state == kDone ? 1 : 0;
}

void Core::shutdown(int cancel_status) {
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (stop_) return;
        stop_ = true;
        const auto now = clk::now();
        for (auto* q : {&small_q_, &large_q_}) {
            for (Job* j : *q) {
                j->status = cancel_status;
                j->state = kDone;
                j->t_done = now;
                latency_ms_.push_back(
                    std::chrono::duration<double, std::milli>(now - j->t_submit).count());
                log_event("cancel", j);
            }
            q->clear();
        }
    }
    cv_work_.notify_all();
    cv_done_.notify_all();
}

bool Core::stopping() {
    std::lock_guard<std::mutex> lk(mu_);
    return stop_;
}

void Core::stats(double* p50, double* p99, int64_t* completed) {
    std::vector<double> v;
    {
        std::lock_guard<std::mutex> lk(mu_);
        v = latency_ms_;
    }
    if (completed) *completed = (int64_t)v.size();
    if (v.empty()) {
        if (p50) *p50 = 0.0;
        if (p99) *p99 = 0.0;
        return;
    }
    std::sort(v.begin(), v.end());
    auto q = [&](double f) {
        const double k = f * (double)(v.size() - 1);
        const size_t lo = (size_t)k, hi = std::min(lo + 1, v.size() - 1);
        return v[lo] + (v[hi] - v[lo]) * (k - (double)lo);
    };
    if (p50) *p50 = q(0.5);
    if (p99) *p99 = q(0.99);
}

Job* Core::next_large(int worker, const FreeBytes& free_bytes, int busy_status) {
    const auto recheck = std::chrono::microseconds(cfg_.recheck_us);
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        if (stop_) return nullptr;
        if (large_q_.empty()) {
            cv_work_.wait(lk);
            continue;
        }
        Job* f = large_q_.front();
        if (f->bytes > cfg_.budget) {  // can never fit: completes at once
            large_q_.pop_front();
            f->worker = worker;
            f->status = busy_status;
            f->state = kDone;
            f->t_start = f->t_done = clk::now();
            latency_ms_.push_back(
                std::chrono::duration<double, std::milli>(f->t_done - f->t_submit).count());
            log_event("busy", f);
            cv_done_.notify_all();
            continue;
        }
        if (used_ + f->bytes > cfg_.budget) {
            cv_work_.wait_for(lk, recheck);
            continue;
        }
        bool fits = f->resident;
        if (!fits) {
            // the memory query is a device call: made without the lock, then the
            // queue is looked at again (another worker may have taken the request)
            lk.unlock();
            const int64_t fr = free_bytes();
            lk.lock();
            if (stop_) return nullptr;
            if (large_q_.empty() || large_q_.front() != f) continue;
            fits = fr > f->bytes + cfg_.margin;
        }
        if (fits && used_ + f->bytes <= cfg_.budget) {
            large_q_.pop_front();
            used_ += f->bytes;
            f->worker = worker;
            f->state = kRunning;
            f->t_start = clk::now();
            log_event("start", f);
            return f;
        }
        cv_work_.wait_for(lk, recheck);
    }
}

int Core::next_small(int worker, int max_jobs, int64_t wait_us, std::vector<Job*>& out) {
    out.clear();
    std::unique_lock<std::mutex> lk(mu_);
    auto ready = [&] { return stop_ || !small_q_.empty(); };
    if (wait_us < 0)
        cv_work_.wait(lk, ready);
    else if (wait_us > 0)
        cv_work_.wait_for(lk, std::chrono::microseconds(wait_us), ready);
    if (stop_) return 0;
    const auto now = clk::now();
    while (!small_q_.empty() && (int)out.size() < max_jobs) {
        Job* j = small_q_.front();
        small_q_.pop_front();
        j->worker = worker;
        j->state = kRunning;
        j->t_start = now;
        log_event("start", j);
        out.push_back(j);
    }
    return (int)out.size();
}

size_t Core::small_waiting() {
    std::lock_guard<std::mutex> lk(mu_);
    return small_q_.size();
}

void Core::complete(Job* j, int status) {
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (!j->small) used_ -= j->bytes;
        j->status = status;
        j->state = kDone;
        j->t_done = clk::now();
        latency_ms_.push_back(
            std::chrono::duration<double, std::milli>(j->t_done - j->t_submit).count());
        log_event("done", j);
    }
    cv_done_.notify_all();
    cv_work_.notify_all();
}

bool Core::visit(uint64_t ticket, const std::function<void(const Job&)>& f) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return false;
    f(*it->second);
    return true;
}

int64_t Core::bytes_in_use() {
    std::lock_guard<std::mutex> lk(mu_);
    return used_;
}

}  // namespace srv
}  // namespace pvi
