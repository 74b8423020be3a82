// tt_server.hip -- many streams on one GPU: admission of streams against one HBM budget and
// continuous batching of their frames at LM-iteration boundaries. The per-frame solve (Sec. 2) is
// the one the single-stream path queues, step for step; only the interleaving of streams differs.
//
// One scheduler thread per server queues the work in rounds. A round takes every frame whose front
// stage (normal map, matching, pre-selection) has completed and that still has LM iterations to go.
// Frames of coupled streams with no stage of their own run the round on the server's HIP stream,
// each stage one multi-system launch over all of them (argument tables written per round); the
// others assemble on their stream's HIP stream and join by events. All coupled systems are factored
// and solved together on the server's HIP stream, each frame takes its update, and a frame that
// has done its last iteration queues its outputs (on its stream's HIP stream) and an event. The thread keeps at
// most `ahead` rounds queued beyond the device, so that a frame whose front stage finishes joins
// within that many rounds, and it notices completions by querying the frames' events between
// rounds.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tt_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

enum { F_QUEUED = 0, F_FRONT = 1, F_ROUNDS = 2, F_TAIL = 3, F_DONE = 4 };

struct Frame {
  uint64_t id = 0;
  tt_stream* s = nullptr;
  tt_frame_device f{};
  Clock::time_point t_submit;
  DevState dd;
  hipEvent_t ev_front = nullptr;  // the stream's front-done event for this frame (not owned)
  hipEvent_t ev_done = nullptr;   // owned (server pool)
  int* err_host = nullptr;        // pinned word: the stream's device error bits after the frame
  int it = 0;                     // LM iterations queued
  int state = F_QUEUED;
  int rc = TT_OK;
  double latency_ms = 0.0;
};

struct Slot {
  uint64_t bytes = 0;
  std::deque<Frame*> q;    // submitted, front not yet queued
  Frame* cur = nullptr;    // front queued or in the rounds (the next frame waits for it)
  int pending = 0;         // frames not yet done
};

}  // namespace

struct tt_server {
  int dev = 0;
  hipStream_t st = nullptr;
  bool own_st = false;
  uint64_t budget = 0, reserved = 0;
  int ahead = 1;
  std::mutex mu;
  std::condition_variable cv;  // every change of state: submissions, completions, releases
  std::deque<uint64_t> admit_q;
  uint64_t next_admit = 1, next_ticket = 1;
  std::unordered_map<tt_stream*, Slot> open;
  std::unordered_map<uint64_t, Frame*> frames;
  bool stop = false;
  int64_t submitted = 0, done = 0, rounds = 0, frame_iters = 0;
  // pools (guarded by mu)
  std::vector<hipEvent_t> ev_free;
  std::vector<int*> pin_free;
  std::vector<int*> pin_blocks;
  // owned by the scheduler thread
  std::vector<Frame*> fronting, active, tailing;
  std::deque<hipEvent_t> inflight_rounds;
  std::vector<hipEvent_t> round_ev_free;
  // argument tables of the rounds' multi-system launches: a ring of pinned staging slots and their
  // device copies, one slot per round (scheduler thread)
  std::vector<void*> tab_host, tab_dev;
  size_t tab_cap = 0;  // bytes per slot
  size_t tab_next = 0;
  std::thread worker;
};

namespace {

constexpr int kPinBlock = 1024;

// A pinned word and an event for a new frame (mu held).
int take_resources(tt_server* sv, Frame* fr) {
  if (sv->pin_free.empty()) {
    int* blk = nullptr;
    if (hipHostMalloc((void**)&blk, sizeof(int) * kPinBlock, 0) != hipSuccess) return TT_ENOMEM;
    sv->pin_blocks.push_back(blk);
    for (int i = 0; i < kPinBlock; i++) sv->pin_free.push_back(blk + i);
  }
  if (sv->ev_free.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return TT_EDEVICE;
    sv->ev_free.push_back(e);
  }
  fr->err_host = sv->pin_free.back();
  sv->pin_free.pop_back();
  fr->ev_done = sv->ev_free.back();
  sv->ev_free.pop_back();
  *fr->err_host = 0;
  return TT_OK;
}

void give_back(tt_server* sv, Frame* fr) {
  if (fr->err_host) sv->pin_free.push_back(fr->err_host);
  if (fr->ev_done) sv->ev_free.push_back(fr->ev_done);
  delete fr;
}

// The frame's normal map, matching and pre-selection on its stream's side queue.
int start_front(Frame* fr) {
  tt_stream* s = fr->s;
  fr->dd = ttx::frame_view(s, fr->f.depth, fr->f.feat_xyz, fr->f.feat_desc);
  const int rc = ttx::enqueue_front(s, fr->dd, fr->f.K2, s->st, fr->f.inputs_ready);
  if (rc) return rc;
  fr->ev_front = ttx::front_done_event(s);
  return TT_OK;
}

// Outputs, the device error word (copied, then cleared for the next frame) and the done event.
int end_frame(Frame* fr) {
  tt_stream* s = fr->s;
  int rc = ttx::enqueue_frame_end(s, fr->f.out_vertices, fr->f.out_dq, s->st);
  if (rc) return rc;
  if (hipMemcpyAsync(fr->err_host, &s->d.sc->err, sizeof(int), hipMemcpyDeviceToHost, s->st) != hipSuccess ||
      hipMemsetAsync(&s->d.sc->err, 0, sizeof(int), s->st) != hipSuccess ||
      hipEventRecord(fr->ev_done, s->st) != hipSuccess)
    return TT_EDEVICE;
  return TT_OK;
}

void free_tables(tt_server* sv) {
  for (void* h : sv->tab_host) (void)hipHostFree(h);
  for (void* d : sv->tab_dev) (void)hipFree(d);
  sv->tab_host.clear();
  sv->tab_dev.clear();
  sv->tab_cap = 0;
}

// A slot of at least `bytes` for this round's tables. The ring has ahead + 2 slots: the scheduler
// keeps at most `ahead` rounds queued beyond the device and waits for older ones, so a slot's
// staging copy has run before the slot comes round again (and the device copy is written on the
// server's queue, behind every earlier round that reads it). Growing waits for the queue first.
int table_slot(tt_server* sv, size_t bytes, void** host, void** dev) {
  const size_t nslot = (size_t)sv->ahead + 2;
  if (bytes > sv->tab_cap || sv->tab_host.size() != nslot) {
    if (hipStreamSynchronize(sv->st) != hipSuccess) return TT_EDEVICE;
    free_tables(sv);
    const size_t cap = std::max<size_t>((bytes + 65535) / 65536 * 65536, 65536);
    for (size_t i = 0; i < nslot; i++) {
      void *h = nullptr, *d = nullptr;
      if (hipHostMalloc(&h, cap, 0) != hipSuccess) return TT_ENOMEM;
      sv->tab_host.push_back(h);
      if (hipMalloc(&d, cap) != hipSuccess) return TT_ENOMEM;
      sv->tab_dev.push_back(d);
    }
    sv->tab_cap = cap;
  }
  const size_t i = sv->tab_next++ % nslot;
  *host = sv->tab_host[i];
  *dev = sv->tab_dev[i];
  return TT_OK;
}

// The tables of the frames entering the rounds (m0) and of those continuing (m1), written to a
// slot and copied to the device on the server's queue.
int write_tables(tt_server* sv, const std::vector<Frame*>& m0, const std::vector<Frame*>& m1, LMMulti* t0,
                 LMMulti* t1) {
  const size_t b0 = (lm_multi_bytes((int)m0.size()) + 255) / 256 * 256, b1 = lm_multi_bytes((int)m1.size());
  void *h = nullptr, *d = nullptr;
  int rc = table_slot(sv, b0 + b1, &h, &d);
  if (rc) return rc;
  const std::vector<Frame*>* grp[2] = {&m0, &m1};
  LMMulti* tab[2] = {t0, t1};
  const size_t off[2] = {0, b0};
  for (int k = 0; k < 2; k++) {
    if (grp[k]->empty()) continue;
    std::vector<DevState*> ds;
    std::vector<const tt_params*> ps;
    std::vector<Intr> ks;
    for (Frame* fr : *grp[k]) {
      ds.push_back(&fr->dd);
      ps.push_back(&fr->s->P);
      ks.push_back(ttx::intr(fr->s));
    }
    if (lm_multi_fill(ds.data(), ps.data(), ks.data(), (int)ds.size(), static_cast<char*>(h) + off[k],
                      static_cast<char*>(d) + off[k], tab[k]) != hipSuccess)
      return TT_EDEVICE;
  }
  return hipMemcpyAsync(d, h, b0 + b1, hipMemcpyHostToDevice, sv->st) == hipSuccess ? TT_OK : TT_EDEVICE;
}

// Work queued on queue `from` so far runs before work queued on `to` from now on.
int order_after(tt_stream* s, hipStream_t from, hipStream_t to) {
  hipEvent_t ev = nullptr;
  if (ttx::ev_sync_get(s, &ev) != hipSuccess) return TT_EDEVICE;
  const bool good = hipEventRecord(ev, from) == hipSuccess && hipStreamWaitEvent(to, ev, 0) == hipSuccess;
  ttx::ev_sync_put(s, ev);
  return good ? TT_OK : TT_EDEVICE;
}

// One LM-iteration round over the frames in sv->active (scheduler thread, mu not held). Frames that
// fail to queue, and frames done with their iterations, move to `out` (state F_TAIL, rc set).
// Frames of streams whose stages can run as multi-system launches run the whole round on the
// server's queue, one launch per stage for all of them; the others assemble and update on their
// own stream's queue.
int queue_round(tt_server* sv, std::vector<Frame*>& out) {
  std::vector<Frame*> act;
  act.swap(sv->active);
  std::vector<Frame*> keep;
  auto fail = [&](Frame* fr, int rc) {
    fr->rc = rc;
    fr->state = F_TAIL;
    out.push_back(fr);
  };
  // entering frames: LM set-up (multi-system frames: in the round's launch below); frames with no
  // iterations end here
  auto multi = [](const Frame* fr) { return ttx::multi_ok(fr->s) && fr->s->P.lm_iters > 0; };
  std::vector<Frame*> work;
  for (Frame* fr : act) {
    if (fr->it == 0 && !multi(fr)) {
      const int rc = ttx::enqueue_lm_begin(fr->s, fr->s->st);
      if (rc) {
        fail(fr, rc);
        continue;
      }
    }
    if (fr->it >= fr->s->P.lm_iters) {
      const int rc = end_frame(fr);
      if (rc) fail(fr, rc);
      else {
        fr->state = F_TAIL;
        out.push_back(fr);
      }
      continue;
    }
    work.push_back(fr);
  }
  // the other frames assemble on their own queues (per-node solver streams also solve there)
  std::vector<Frame*> m0, m1, coupled, ok;
  for (Frame* fr : work) {
    if (multi(fr)) {
      (fr->it == 0 ? m0 : m1).push_back(fr);
      continue;
    }
    int rc = ttx::enqueue_assemble(fr->s, fr->dd, fr->it, fr->s->st);
    if (!rc && fr->s->P.solver == TT_SOLVE_NODE) rc = ttx::enqueue_node_solve(fr->s, fr->dd, fr->s->st);
    if (rc) {
      fail(fr, rc);
      continue;
    }
    ok.push_back(fr);
    if (fr->s->P.solver != TT_SOLVE_NODE) coupled.push_back(fr);
  }
  // multi-system frames: those entering the rounds after their front stage and their stream's
  // earlier work; then set-up, assembly and damping on the server's queue, one launch per stage
  LMMulti t0, t1;
  int mrc = TT_OK;
  for (Frame* fr : m0)
    if (!mrc) mrc = order_after(fr->s, fr->s->st, sv->st);
  if (!m0.empty() || !m1.empty()) {
    if (!mrc) mrc = write_tables(sv, m0, m1, &t0, &t1);
    if (!mrc && t0.jobs &&
        (launch_lm_multi_begin(t0, sv->st) != hipSuccess || launch_lm_multi_assemble(t0, 0, sv->st) != hipSuccess))
      mrc = TT_EDEVICE;
    if (!mrc && t1.jobs && launch_lm_multi_assemble(t1, 1, sv->st) != hipSuccess) mrc = TT_EDEVICE;
    std::vector<DevState*> ir;
    for (Frame* fr : m0)
      if (fr->s->d.prec != TT_FP32) ir.push_back(&fr->dd);
    for (Frame* fr : m1)
      if (fr->s->d.prec != TT_FP32) ir.push_back(&fr->dd);
    if (!mrc && !ir.empty() && launch_ir_prepare_batch(ir.data(), (int)ir.size(), sv->st) != hipSuccess)
      mrc = TT_EDEVICE;
  }
  // the coupled frames on their own queues before the server's queue; every coupled system
  // factored and solved in one batched launch there
  int brc = TT_OK;
  for (Frame* fr : coupled)
    if (!brc) brc = order_after(fr->s, fr->s->st, sv->st);
  std::vector<tt_stream*> ss;
  std::vector<DevState*> dp;
  for (Frame* fr : coupled) {
    ss.push_back(fr->s);
    dp.push_back(&fr->dd);
  }
  if (!mrc)
    for (const std::vector<Frame*>* g : {&m0, &m1})
      for (Frame* fr : *g) {
        ss.push_back(fr->s);
        dp.push_back(&fr->dd);
      }
  if (!brc && !ss.empty()) brc = ttx::enqueue_solve(ss.data(), dp.data(), (int)ss.size(), sv->st);
  if (!brc && !coupled.empty()) {  // back to the coupled frames' own queues
    hipEvent_t ev = nullptr;
    if (ttx::ev_sync_get(coupled[0]->s, &ev) != hipSuccess) {
      brc = TT_EDEVICE;
    } else {
      if (hipEventRecord(ev, sv->st) != hipSuccess) brc = TT_EDEVICE;
      for (Frame* fr : coupled)
        if (!brc && hipStreamWaitEvent(fr->s->st, ev, 0) != hipSuccess) brc = TT_EDEVICE;
      ttx::ev_sync_put(coupled[0]->s, ev);
    }
  }
  if (!mrc) mrc = brc;
  // multi-system frames: candidate, cost, accept / reject
  if (!mrc && t0.jobs && launch_lm_multi_finish(t0, sv->st) != hipSuccess) mrc = TT_EDEVICE;
  if (!mrc && t1.jobs && launch_lm_multi_finish(t1, sv->st) != hipSuccess) mrc = TT_EDEVICE;
  for (Frame* fr : ok) {
    if (brc && fr->s->P.solver != TT_SOLVE_NODE) {
      fail(fr, brc);
      continue;
    }
    int rc = ttx::enqueue_finish(fr->s, fr->dd, fr->s->st);
    if (rc) {
      fail(fr, rc);
      continue;
    }
    fr->it += 1;
    if (fr->it >= fr->s->P.lm_iters) {
      rc = end_frame(fr);
      if (rc) fail(fr, rc);
      else {
        fr->state = F_TAIL;
        out.push_back(fr);
      }
    } else {
      keep.push_back(fr);
    }
  }
  for (const std::vector<Frame*>* g : {&m0, &m1})
    for (Frame* fr : *g) {
      if (mrc) {
        fail(fr, mrc);
        continue;
      }
      fr->it += 1;
      if (fr->it < fr->s->P.lm_iters) {
        keep.push_back(fr);
        continue;
      }
      // outputs on the stream's own queue, after the server's queue
      int rc = order_after(fr->s, sv->st, fr->s->st);
      if (!rc) rc = end_frame(fr);
      if (rc) fail(fr, rc);
      else {
        fr->state = F_TAIL;
        out.push_back(fr);
      }
    }
  sv->rounds += 1;
  sv->frame_iters += (int64_t)work.size();
  sv->active.swap(keep);
  // bound the rounds queued beyond the device
  hipEvent_t rev = nullptr;
  if (!sv->round_ev_free.empty()) {
    rev = sv->round_ev_free.back();
    sv->round_ev_free.pop_back();
  } else if (hipEventCreateWithFlags(&rev, hipEventDisableTiming) != hipSuccess) {
    return TT_EDEVICE;
  }
  if (hipEventRecord(rev, sv->st) != hipSuccess) return TT_EDEVICE;
  sv->inflight_rounds.push_back(rev);
  while ((int)sv->inflight_rounds.size() > sv->ahead) {
    hipEvent_t e = sv->inflight_rounds.front();
    sv->inflight_rounds.pop_front();
    (void)hipEventSynchronize(e);
    sv->round_ev_free.push_back(e);
  }
  return TT_OK;
}

void scheduler(tt_server* sv) {
  (void)hipSetDevice(sv->dev);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // streams whose previous frame is fully queued take their next frame
    std::vector<Frame*> starting;
    for (auto& kv : sv->open) {
      Slot& sl = kv.second;
      if (!sl.cur && !sl.q.empty()) {
        Frame* fr = sl.q.front();
        sl.q.pop_front();
        sl.cur = fr;
        fr->state = F_FRONT;
        starting.push_back(fr);
      }
    }
    const bool idle = starting.empty() && sv->fronting.empty() && sv->active.empty() && sv->tailing.empty();
    if (idle) {
      if (sv->stop) break;
      sv->cv.wait(lk);
      continue;
    }
    lk.unlock();
    std::vector<Frame*> moved;  // frames whose front stage was queued, joined or that left the rounds
    for (Frame* fr : starting) {
      const int rc = start_front(fr);
      if (rc) {
        fr->rc = rc;
        fr->state = F_TAIL;
        sv->tailing.push_back(fr);
      } else {
        sv->fronting.push_back(fr);
      }
    }
    // fronts that have completed join this round
    for (size_t i = 0; i < sv->fronting.size();) {
      Frame* fr = sv->fronting[i];
      const hipError_t q = hipEventQuery(fr->ev_front);
      if (q == hipSuccess || q != hipErrorNotReady) {
        sv->fronting.erase(sv->fronting.begin() + (long)i);
        if (q == hipSuccess) {
          fr->state = F_ROUNDS;
          sv->active.push_back(fr);
        } else {
          fr->rc = TT_EDEVICE;
          fr->state = F_TAIL;
          sv->tailing.push_back(fr);
        }
      } else {
        i++;
      }
    }
    bool progressed = false;
    if (!sv->active.empty()) {
      std::vector<Frame*> left;
      const int rc = queue_round(sv, left);
      for (Frame* fr : left) {
        if (rc && !fr->rc) fr->rc = rc;
        sv->tailing.push_back(fr);
        moved.push_back(fr);
      }
      progressed = true;
    }
    // completions
    std::vector<Frame*> finished;
    for (size_t i = 0; i < sv->tailing.size();) {
      Frame* fr = sv->tailing[i];
      hipError_t q = hipSuccess;
      if (fr->rc == TT_OK) q = hipEventQuery(fr->ev_done);
      if (q == hipErrorNotReady) {
        i++;
        continue;
      }
      if (q != hipSuccess) fr->rc = TT_EDEVICE;
      else if (fr->rc == TT_OK && *fr->err_host != 0) fr->rc = TT_EDEVICE;
      fr->latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - fr->t_submit).count();
      finished.push_back(fr);
      sv->tailing.erase(sv->tailing.begin() + (long)i);
    }
    lk.lock();
    for (Frame* fr : moved) {
      auto it = sv->open.find(fr->s);
      if (it != sv->open.end() && it->second.cur == fr) it->second.cur = nullptr;  // its next frame may start
    }
    for (Frame* fr : sv->tailing) {  // failed before joining: release the stream too
      auto it = sv->open.find(fr->s);
      if (it != sv->open.end() && it->second.cur == fr) it->second.cur = nullptr;
    }
    for (Frame* fr : finished) {
      auto it = sv->open.find(fr->s);
      if (it != sv->open.end()) {
        if (it->second.cur == fr) it->second.cur = nullptr;
        it->second.pending -= 1;
      }
      fr->state = F_DONE;
      sv->done += 1;
    }
    if (!finished.empty() || !moved.empty()) sv->cv.notify_all();
    if (!progressed && finished.empty() && starting.empty())
      sv->cv.wait_for(lk, std::chrono::microseconds(20));  // only fronts or tails in flight
  }
}

}  // namespace

extern "C" {

void tt_server_default_params(tt_server_params* p) {
  if (!p) return;
  p->hbm_budget_bytes = 0;
  p->max_rounds_ahead = 1;
}

int tt_server_create(const tt_server_params* p, void* hip_stream, tt_server** out) {
  if (!p || !out || p->max_rounds_ahead < 0 || p->max_rounds_ahead > 8) return TT_EINVAL;
  *out = nullptr;
  tt_server* sv = new (std::nothrow) tt_server();
  if (!sv) return TT_ENOMEM;
  if (hipGetDevice(&sv->dev) != hipSuccess) {
    delete sv;
    return TT_EDEVICE;
  }
  sv->budget = p->hbm_budget_bytes;
  sv->ahead = p->max_rounds_ahead ? p->max_rounds_ahead : 1;
  if (hip_stream) {
    sv->st = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&sv->st, hipStreamNonBlocking) != hipSuccess) {
      delete sv;
      return TT_EDEVICE;
    }
    sv->own_st = true;
  }
  try {
    sv->worker = std::thread(scheduler, sv);
  } catch (...) {
    if (sv->own_st) (void)hipStreamDestroy(sv->st);
    delete sv;
    return TT_ENOMEM;
  }
  *out = sv;
  return TT_OK;
}

int tt_server_open(tt_server* sv, const tt_params* p, const tt_intrinsics* K, const float* pts_xyz, int M,
                   const float* feat_xyz, const uint8_t* feat_desc, int K1, int K2max, double wait_s,
                   tt_stream** out) {
  if (!sv || !p || !K || !out || K2max < 0 || K2max > (1 << 23) || !(wait_s >= 0.0)) return TT_EINVAL;
  *out = nullptr;
  const auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(
                                           std::min(wait_s, 1e6)));
  std::unique_lock<std::mutex> lk(sv->mu);
  const uint64_t me = sv->next_admit++;
  sv->admit_q.push_back(me);
  auto leave = [&](int rc) {
    sv->admit_q.erase(std::find(sv->admit_q.begin(), sv->admit_q.end(), me));
    sv->cv.notify_all();
    return rc;
  };
  for (;;) {
    // our turn, and some room
    const bool ready = sv->cv.wait_until(lk, deadline, [&] {
      return sv->admit_q.front() == me && (sv->budget == 0 || sv->reserved < sv->budget);
    });
    if (!ready) return leave(TT_EBUSY);
    const uint64_t room = sv->budget ? sv->budget - sv->reserved : 0;
    const uint64_t held = sv->reserved;
    lk.unlock();
    tt_params q = *p;
    if (sv->budget) q.hbm_budget_bytes = p->hbm_budget_bytes ? std::min<uint64_t>(p->hbm_budget_bytes, room) : room;
    tt_stream* s = nullptr;
    int rc = tt_create_stream(&q, K, nullptr, &s);
    if (!rc) rc = tt_set_template(s, pts_xyz, M, feat_xyz, feat_desc, K1);
    if (!rc && K2max > 0) rc = ttx::ensure_k2(s, K2max);
    uint64_t bytes = 0;
    if (!rc) rc = tt_device_bytes(s, &bytes);
    if (rc && s) {
      (void)tt_destroy(s);
      s = nullptr;
    }
    lk.lock();
    if (!rc) {
      s->served.store(true);  // owned by the server until tt_server_close
      Slot& sl = sv->open[s];
      sl.bytes = bytes;
      sv->reserved += bytes;
      *out = s;
      return leave(TT_OK);
    }
    if (rc != TT_ENOMEM || sv->budget == 0 || held == 0) return leave(rc);
    // it did not fit next to the streams open now: wait until one of them releases its bytes
    const bool freed = sv->cv.wait_until(lk, deadline, [&] { return sv->reserved < held; });
    if (!freed) return leave(TT_EBUSY);
  }
}

int tt_server_submit(tt_server* sv, tt_stream* s, const tt_frame_device* f, uint64_t* ticket) {
  if (!sv || !s || !f || !ticket || !f->depth || f->K2 < 0 || (f->K2 > 0 && (!f->feat_xyz || !f->feat_desc)))
    return TT_EINVAL;
  if (f->K2 > 0 && (uintptr_t)f->feat_desc % 16 != 0) return TT_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  auto it = sv->open.find(s);
  if (it == sv->open.end() || sv->stop) return TT_EINVAL;
  if (f->K2 > s->d.K2cap) return TT_EINVAL;  // beyond the K2max the stream was opened with
  Frame* fr = new (std::nothrow) Frame();
  if (!fr) return TT_ENOMEM;
  const int rc = take_resources(sv, fr);
  if (rc) {
    give_back(sv, fr);
    return rc;
  }
  fr->id = sv->next_ticket++;
  fr->s = s;
  fr->f = *f;
  fr->t_submit = Clock::now();
  it->second.q.push_back(fr);
  it->second.pending += 1;
  sv->frames[fr->id] = fr;
  sv->submitted += 1;
  *ticket = fr->id;
  sv->cv.notify_all();
  return TT_OK;
}

static int report(tt_server* sv, std::unordered_map<uint64_t, Frame*>::iterator it, double* latency_ms) {
  Frame* fr = it->second;
  const int rc = fr->rc;
  if (latency_ms) *latency_ms = fr->latency_ms;
  sv->frames.erase(it);
  give_back(sv, fr);
  return rc;
}

int tt_server_poll(tt_server* sv, uint64_t ticket, int* done, double* latency_ms) {
  if (!sv || !done) return TT_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  auto it = sv->frames.find(ticket);
  if (it == sv->frames.end()) return TT_EINVAL;
  if (it->second->state != F_DONE) {
    *done = 0;
    return TT_OK;
  }
  *done = 1;
  return report(sv, it, latency_ms);
}

int tt_server_wait(tt_server* sv, uint64_t ticket, double wait_s, double* latency_ms) {
  if (!sv || !(wait_s >= 0.0)) return TT_EINVAL;
  const auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(
                                           std::min(wait_s, 1e6)));
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->frames.find(ticket) == sv->frames.end()) return TT_EINVAL;
  // looked up afresh on every wake-up: another thread may collect the report meanwhile
  if (!sv->cv.wait_until(lk, deadline, [&] {
        auto jt = sv->frames.find(ticket);
        return jt == sv->frames.end() || jt->second->state == F_DONE;
      }))
    return TT_EBUSY;
  auto it = sv->frames.find(ticket);
  if (it == sv->frames.end()) return TT_EINVAL;
  return report(sv, it, latency_ms);
}

int tt_server_close(tt_server* sv, tt_stream* s) {
  if (!sv || !s) return TT_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->open.find(s);
  if (it == sv->open.end()) return TT_EINVAL;
  sv->cv.wait(lk, [&] {
    auto jt = sv->open.find(s);
    return jt != sv->open.end() && jt->second.pending == 0;
  });
  it = sv->open.find(s);
  const uint64_t bytes = it->second.bytes;
  sv->open.erase(it);
  // forget reports nobody collected for this stream
  for (auto ft = sv->frames.begin(); ft != sv->frames.end();) {
    if (ft->second->s == s) {
      give_back(sv, ft->second);
      ft = sv->frames.erase(ft);
    } else {
      ++ft;
    }
  }
  lk.unlock();
  s->served.store(false);
  const int rc = tt_destroy(s);
  lk.lock();
  sv->reserved -= bytes;
  sv->cv.notify_all();
  return rc;
}

int tt_server_get_stats(tt_server* sv, tt_server_stats* out) {
  if (!sv || !out) return TT_EINVAL;
  std::lock_guard<std::mutex> g(sv->mu);
  out->streams_open = (int)sv->open.size();
  out->opens_waiting = (int)sv->admit_q.size();
  out->reserved_bytes = sv->reserved;
  out->frames_submitted = sv->submitted;
  out->frames_done = sv->done;
  out->rounds = sv->rounds;
  out->frame_iterations = sv->frame_iters;
  return TT_OK;
}

int tt_server_destroy(tt_server* sv) {
  if (!sv) return TT_EINVAL;
  std::vector<tt_stream*> streams;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv.wait(lk, [&] { return sv->done == sv->submitted; });
    for (auto& kv : sv->open) streams.push_back(kv.first);
  }
  int rc = TT_OK;
  for (tt_stream* s : streams) {
    const int r = tt_server_close(sv, s);
    if (r && !rc) rc = r;
  }
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
    sv->cv.notify_all();
  }
  sv->worker.join();
  for (hipEvent_t e : sv->inflight_rounds) {
    (void)hipEventSynchronize(e);
    (void)hipEventDestroy(e);
  }
  for (hipEvent_t e : sv->round_ev_free) (void)hipEventDestroy(e);
  (void)hipStreamSynchronize(sv->st);
  free_tables(sv);
  for (auto& kv : sv->frames) give_back(sv, kv.second);
  sv->frames.clear();
  for (hipEvent_t e : sv->ev_free) (void)hipEventDestroy(e);
  for (int* b : sv->pin_blocks) (void)hipHostFree(b);
  if (sv->own_st && sv->st) (void)hipStreamDestroy(sv->st);
  delete sv;
  return rc;
}

}  // extern "C"
