// Native load generator for the serving path (include/memshield_serve.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "memshield.h"
#include "memshield_resident.h"
#include "memshield_serve.h"
#include "ms_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

void wait_until(Clock::time_point t) {
  for (;;) {
    const auto now = Clock::now();
    if (now >= t) return;
    const auto left = t - now;
    if (left > std::chrono::microseconds(300))
      std::this_thread::sleep_for(left - std::chrono::microseconds(200));
    else
      std::this_thread::yield();
  }
}

double us_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::micro>(b - a).count();
}

ms_request make_request(const ms_serve_trace* tr, uint64_t i,
                        const ms_key* keys, const void* src, void* dst) {
  ms_request r;
  std::memset(&r, 0, sizeof(r));
  r.op = tr->op[i];
  r.client = tr->client[i];
  r.key = keys[tr->client[i]];
  r.src = static_cast<const uint8_t*>(src) + tr->src_page[i] * MS_PAGE_SIZE;
  r.dst = static_cast<uint8_t*>(dst) + tr->dst_page[i] * MS_PAGE_SIZE;
  r.n_pages = tr->n_pages[i];
  r.nonce.kind = MS_NONCE_LINEAR;
  r.nonce.base = tr->va[i];
  r.nonce.stride = MS_PAGE_SIZE;
  r.nonce.tag = tr->pid[i];
  return r;
}

double percentile(std::vector<double>& sorted, double q) {
  if (sorted.empty()) return 0;
  const double pos = q * (sorted.size() - 1);
  const size_t lo = (size_t)pos;
  const size_t hi = std::min(lo + 1, sorted.size() - 1);
  const double f = pos - lo;
  return sorted[lo] * (1 - f) + sorted[hi] * f;
}

}  // namespace

extern "C" ms_status ms_serve_run(ms_ctx* c, const ms_serve_trace* tr,
                                  const ms_key* keys, uint32_t n_keys,
                                  const void* src_pool, uint64_t src_pages,
                                  void* dst_pool, uint64_t dst_pages,
                                  int32_t mode, uint32_t submit_threads,
                                  double* lat_out, ms_serve_result* res) {
  if (!c || !tr || !keys || !res || !src_pool || !dst_pool) return MS_EINVAL;
  if (mode != MS_SERVE_BATCHED && mode != MS_SERVE_PLAIN &&
      mode != MS_SERVE_RESIDENT)
    return MS_EINVAL;
  if (mode == MS_SERVE_RESIDENT && n_keys > MS_RESIDENT_MAX_KEYS)
    return MS_EINVAL;
  if (submit_threads == 0 || submit_threads > 64) return MS_EINVAL;
  const uint64_t n = tr->n;
  for (uint64_t i = 0; i < n; ++i) {
    if (tr->client[i] >= n_keys || tr->n_pages[i] == 0) return MS_EINVAL;
    if (tr->src_page[i] > src_pages || tr->n_pages[i] > src_pages - tr->src_page[i])
      return MS_EINVAL;
    if (tr->dst_page[i] > dst_pages || tr->n_pages[i] > dst_pages - tr->dst_page[i])
      return MS_EINVAL;
    if (i && tr->arrival_s[i] < tr->arrival_s[i - 1]) return MS_EINVAL;
  }
  std::memset(res, 0, sizeof(*res));
  if (n == 0) return MS_OK;

  // resident mode: one engine holding every client's key, one descriptor per
  // page (so a request's pages are ciphered by as many waves at once), as
  // many workers as one workgroup per compute unit allows
  ms_resident* rk = nullptr;
  if (mode == MS_SERVE_RESIDENT) {
    ms_resident_config rc;
    ms_resident_config_default(&rc);
    rc.workers = (uint32_t)ms_internal_cu_count(c) * 4u - 1u;
    rc.desc_pages = 1;
    rc.ring_depth = 1u << 16;
    const ms_status rs = ms_resident_start_keys(c, &rc, keys, n_keys, &rk);
    if (rs != MS_OK) return rs;
  }

  // Warm-up before the clock starts: request 0's first page, through the
  // mode's own path, so that one-time costs (the serving stage's start, the
  // first launch) do not land on the first arrivals.  The page it writes is
  // written again by request 0.
  {
    ms_request w = make_request(tr, 0, keys, src_pool, dst_pool);
    w.n_pages = 1;
    ms_status ws = MS_OK;
    if (mode == MS_SERVE_PLAIN) {
      ws = (w.op == MS_DECRYPT)
               ? ms_decrypt_pages(c, w.key, w.src, w.dst, 1, &w.nonce, nullptr)
               : ms_encrypt_pages(c, w.key, w.src, w.dst, 1, &w.nonce, nullptr);
      if (ws == MS_OK && hipDeviceSynchronize() != hipSuccess) ws = MS_EDEVICE;
    } else {
      ms_ticket tk = 0;
      int32_t dn = 0;
      ws = rk ? ms_resident_submit_keyed(rk, tr->client[0], w.src, w.dst, 1,
                                         &w.nonce, &tk)
              : ms_submit(c, &w, 1, &tk);
      if (ws == MS_OK)
        ws = rk ? ms_resident_poll(rk, &tk, 1, &dn, 10000000000ull)
                : ms_poll(c, &tk, 1, &dn, 10000000000ull);
      if (ws == MS_OK && dn != 1) ws = dn < 0 ? (ms_status)dn : MS_EDEVICE;
    }
    if (ws != MS_OK) {
      if (rk) (void)ms_resident_stop(rk);
      return ws;
    }
  }

  std::vector<Clock::time_point> done_t(n);
  std::vector<double> late(n, 0.0);
  std::vector<double> call_us(n, 0.0);  // time inside the submitting call
  std::vector<int32_t> state(n, 0);
  std::atomic<uint64_t> retries{0};
  std::atomic<int32_t> fail{0};
  const auto t0 = Clock::now() + std::chrono::milliseconds(20);
  auto arrival = [&](uint64_t i) {
    return t0 + std::chrono::duration_cast<Clock::duration>(
                    std::chrono::duration<double>(tr->arrival_s[i]));
  };
  ms_status st = MS_OK;

  if (mode == MS_SERVE_BATCHED || mode == MS_SERVE_RESIDENT) {
    auto submit_one = [&](uint64_t i, const ms_request& r, ms_ticket* tk) {
      if (rk)
        return ms_resident_submit_keyed(rk, tr->client[i], r.src, r.dst,
                                        r.n_pages, &r.nonce, tk);
      return ms_submit(c, &r, 1, tk);
    };
    auto poll_some = [&](const ms_ticket* t, size_t m, int32_t* dn) {
      return rk ? ms_resident_poll(rk, t, m, dn, 0) : ms_poll(c, t, m, dn, 0);
    };
    std::mutex mu;
    std::vector<std::pair<uint64_t, ms_ticket>> fresh;
    std::atomic<uint32_t> submitters_done{0};
    auto submitter = [&](uint32_t t) {
      for (uint64_t i = t; i < n && !fail.load(); i += submit_threads) {
        wait_until(arrival(i));
        late[i] = us_between(arrival(i), Clock::now());
        ms_request r = make_request(tr, i, keys, src_pool, dst_pool);
        ms_ticket tk = 0;
        const auto c0 = Clock::now();
        for (;;) {
          const ms_status s = submit_one(i, r, &tk);
          if (s == MS_OK) break;
          if (s != MS_EAGAIN) {
            fail.store(s);
            break;
          }
          retries.fetch_add(1);
          std::this_thread::yield();
        }
        if (fail.load()) break;
        call_us[i] = us_between(c0, Clock::now());
        std::lock_guard<std::mutex> lk(mu);
        fresh.emplace_back(i, tk);
      }
      submitters_done.fetch_add(1);
    };
    std::vector<std::thread> th;
    for (uint32_t t = 0; t < submit_threads; ++t) th.emplace_back(submitter, t);
    // poller: observe completions
    std::vector<std::pair<uint64_t, ms_ticket>> pend;
    std::vector<ms_ticket> tks;
    std::vector<int32_t> dn;
    uint64_t observed = 0;
    Clock::time_point last_arrival = arrival(n - 1);
    while (observed < n && !fail.load()) {
      // read before taking the fresh tickets: a submitter pushes its last
      // ticket before it counts itself done, so once all are counted here
      // the merge below holds every ticket (read after the merge, a ticket
      // pushed in between would be lost)
      const bool all_submitted = submitters_done.load() == submit_threads;
      {
        std::lock_guard<std::mutex> lk(mu);
        pend.insert(pend.end(), fresh.begin(), fresh.end());
        fresh.clear();
      }
      if (pend.empty()) {
        if (all_submitted) break;
        std::this_thread::yield();
        continue;
      }
      tks.resize(pend.size());
      dn.resize(pend.size());
      for (size_t k = 0; k < pend.size(); ++k) tks[k] = pend[k].second;
      const ms_status ps = poll_some(tks.data(), tks.size(), dn.data());
      if (ps != MS_OK && ps != MS_ETIMEDOUT) {
        fail.store(ps);
        break;
      }
      const auto now = Clock::now();
      size_t w = 0;
      for (size_t k = 0; k < pend.size(); ++k) {
        if (dn[k] != 0) {
          done_t[pend[k].first] = now;
          state[pend[k].first] = dn[k];
          ++observed;
        } else {
          pend[w++] = pend[k];
        }
      }
      pend.resize(w);
      if (now > last_arrival + std::chrono::seconds(60)) {
        st = MS_ETIMEDOUT;
        fail.store(MS_ETIMEDOUT);
        break;
      }
      if (w) std::this_thread::yield();
    }
    for (auto& t : th) t.join();
    if (rk) {
      const ms_status ss = ms_resident_stop(rk);
      if (ss != MS_OK && !fail.load()) fail.store(ss);
    }
    if (fail.load()) {
      if (!rk) (void)ms_drain(c, 60ull * 1000000000ull);
      return st ? st : (ms_status)fail.load();
    }
  } else {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
      return MS_EDEVICE;
    const uint64_t E = 4096;
    std::vector<hipEvent_t> ev(E, nullptr);
    bool ok = true;
    for (auto& e : ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        ok = false;
    std::atomic<uint64_t> issued{0}, completed{0};
    std::thread poller([&] {
      uint64_t j = 0;
      const auto limit = arrival(n - 1) + std::chrono::seconds(60);
      while (j < n && !fail.load()) {
        if (j >= issued.load(std::memory_order_acquire)) {
          std::this_thread::yield();
          continue;
        }
        const hipError_t q = hipEventQuery(ev[j % E]);
        if (q == hipErrorNotReady) {
          if (Clock::now() > limit) {
            fail.store(MS_ETIMEDOUT);
            break;
          }
          std::this_thread::yield();
          continue;
        }
        done_t[j] = Clock::now();
        state[j] = q == hipSuccess ? 1 : MS_EDEVICE;
        ++j;
        completed.store(j, std::memory_order_release);
      }
    });
    for (uint64_t i = 0; ok && i < n && !fail.load(); ++i) {
      while (i >= completed.load(std::memory_order_acquire) + E &&
             !fail.load())
        std::this_thread::yield();
      wait_until(arrival(i));
      late[i] = us_between(arrival(i), Clock::now());
      ms_request r = make_request(tr, i, keys, src_pool, dst_pool);
      const auto c0 = Clock::now();
      ms_status ps =
          (r.op == MS_DECRYPT)
              ? ms_decrypt_pages(c, r.key, r.src, r.dst, r.n_pages, &r.nonce, s)
              : ms_encrypt_pages(c, r.key, r.src, r.dst, r.n_pages, &r.nonce, s);
      if (ps != MS_OK || hipEventRecord(ev[i % E], s) != hipSuccess) {
        fail.store(ps != MS_OK ? ps : MS_EDEVICE);
        break;
      }
      call_us[i] = us_between(c0, Clock::now());
      issued.store(i + 1, std::memory_order_release);
    }
    poller.join();
    (void)hipStreamSynchronize(s);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(s);
    if (!ok) return MS_EDEVICE;
    if (fail.load()) return (ms_status)fail.load();
  }

  std::vector<double> lat(n);
  Clock::time_point last = t0;
  uint64_t bytes = 0;
  for (uint64_t i = 0; i < n; ++i) {
    lat[i] = us_between(arrival(i), done_t[i]);
    if (done_t[i] > last) last = done_t[i];
    bytes += tr->n_pages[i] * MS_PAGE_SIZE;
    if (state[i] != 1) {
      if (!res->failed) {
        res->first_failed = i + 1;
        res->first_failed_state = state[i];
      }
      res->failed++;
    }
    res->late_submit_us_max = std::max(res->late_submit_us_max, late[i]);
  }
  if (lat_out) std::memcpy(lat_out, lat.data(), n * sizeof(double));
  const double wall = std::chrono::duration<double>(last - arrival(0)).count();
  std::vector<double> srt = lat;
  std::sort(srt.begin(), srt.end());
  double sum = 0;
  for (double v : srt) sum += v;
  res->wall_s = wall;
  res->data_gbps = wall > 0 ? bytes / wall / 1e9 : 0;
  res->mean_us = sum / n;
  res->p50_us = percentile(srt, 0.50);
  res->p90_us = percentile(srt, 0.90);
  res->p99_us = percentile(srt, 0.99);
  res->p999_us = percentile(srt, 0.999);
  res->max_us = srt.back();
  res->completed = n;
  res->eagain_retries = retries.load();
  std::sort(call_us.begin(), call_us.end());
  res->submit_call_p50_us = percentile(call_us, 0.50);
  res->submit_call_p99_us = percentile(call_us, 0.99);
  return MS_OK;
}
