// Continuously batched solve server (see server.h for the model).
#include "server.h"

#include <algorithm>
#include <cstring>

namespace crk {

namespace {

size_t lane_footprint(Hierarchy* H, const crk_server_params& p) {
  const size_t stage = sizeof(double2) * 12 * size_t(H->V(0)) * size_t(p.slots_per_lane);
  return mg_solve_footprint(H, p.slots_per_lane, p.solve.form, p.solve) + stage;
}

}  // namespace

Server::Server(const crk_server_params& p) : p_(p), t0_(std::chrono::steady_clock::now()) {
  CRK_REQUIRE(p.slots_per_lane >= 1 && p.slots_per_lane <= 64, "slots_per_lane must be in [1, 64]");
  CRK_REQUIRE(p.max_lanes >= 1 && p.max_lanes <= 16, "max_lanes must be in [1, 16]");
  CRK_REQUIRE(p.idle_ms >= 0, "idle_ms must be >= 0");
  CRK_HIP(hipGetDevice(&device_));
  if (p.hbm_budget_bytes > 0) {
    budget_ = size_t(p.hbm_budget_bytes);
  } else {
    budget_ = device_free_bytes() / 10 * 8;
  }
}

double Server::now() const {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
}

int Server::add(Hierarchy* H) {
  CRK_REQUIRE(H != nullptr, "hierarchy is NULL");
  std::lock_guard<std::mutex> lk(mu_);
  CRK_REQUIRE(!stop_, "server is shutting down");
  auto e = std::make_unique<LatticeEntry>();
  e->H = H;
  e->lane_bytes = lane_footprint(H, p_);
  if (e->lane_bytes > budget_)
    fail(CRK_ENOMEM, "one lane of this lattice (" + std::to_string(e->lane_bytes) +
                         " bytes) does not fit in the server's HBM budget (" + std::to_string(budget_) + ")");
  H->refs++;
  lat_.push_back(std::move(e));
  return int(lat_.size()) - 1;
}

uint64_t Server::submit(int lattice, const double* b, double* x, int nrhs) {
  CRK_REQUIRE(b != nullptr && x != nullptr, "b and x must not be NULL");
  CRK_REQUIRE(nrhs >= 1 && nrhs <= p_.slots_per_lane, "nrhs must be in [1, slots_per_lane]");
  std::lock_guard<std::mutex> lk(mu_);
  CRK_REQUIRE(!stop_, "server is shutting down");
  CRK_REQUIRE(lattice >= 0 && lattice < int(lat_.size()), "unknown lattice id");
  auto r = std::make_unique<Request>();
  r->id = next_id_++;
  r->lattice = lattice;
  r->b = b;
  r->x = x;
  r->nrhs = nrhs;
  r->t_submit = now();
  Request* rp = r.get();
  req_[rp->id] = std::move(r);
  lat_[lattice]->pending.push_back(rp);
  st_.submitted++;
  open_lanes_locked();
  cv_.notify_all();
  return rp->id;
}

// Opens lanes for lattices whose queued RHS exceed the free slots of their
// lanes, while the budget allows, and reaps lanes whose threads have ended.
void Server::open_lanes_locked() {
  for (auto& ep : lat_) {
    LatticeEntry& e = *ep;
    int queued = 0, free = 0;
    for (Request* r : e.pending) queued += r->nrhs - r->started;
    for (Lane* l : e.lanes) free += l->free_slots;
    while (queued > free && int(e.lanes.size()) < p_.max_lanes &&
           size_t(st_.bytes_in_use) + e.lane_bytes <= budget_) {
      Lane* ln = new Lane();
      ln->srv = this;
      ln->lattice = int(&ep - &lat_[0]);
      ln->entry = &e;
      ln->id = e.next_lane_id++;
      ln->bytes = e.lane_bytes;
      ln->free_slots = p_.slots_per_lane;  // reserved until the lane is ready
      ln->idle_since = -1;
      e.lanes.push_back(ln);
      st_.bytes_in_use += int64_t(ln->bytes);
      st_.peak_bytes = std::max(st_.peak_bytes, st_.bytes_in_use);
      st_.lanes_opened++;
      open_lanes_++;
      st_.max_concurrent_lanes = std::max<int64_t>(st_.max_concurrent_lanes, open_lanes_);
      free += p_.slots_per_lane;
      all_lanes_.push_back(ln);
      ln->th = std::thread(lane_main, this, ln);
    }
  }
}

void Server::finish_locked(Request* r) {
  r->done = true;
  r->t_done = now();
  if (r->status == CRK_OK) st_.completed++;
  else st_.failed++;
  done_cv_.notify_all();
}

void Server::fail_pending_locked(int lattice, int code, const std::string& msg) {
  LatticeEntry& e = *lat_[lattice];
  while (!e.pending.empty()) {
    Request* r = e.pending.front();
    e.pending.pop_front();
    r->status = code;
    r->error = msg;
    finish_locked(r);
  }
}

// Removes a lane from its lattice and returns its memory to the budget.
void Server::close_lane_locked(Lane* ln) {
  LatticeEntry& e = *lat_[ln->lattice];
  auto it = std::find(e.lanes.begin(), e.lanes.end(), ln);
  if (it == e.lanes.end()) return;
  e.lanes.erase(it);
  st_.bytes_in_use -= int64_t(ln->bytes);
  st_.lanes_closed++;
  open_lanes_--;
}

bool Server::wait(uint64_t id, double timeout_s, Request& out) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = req_.find(id);
  CRK_REQUIRE(it != req_.end(), "unknown request id");
  Request* r = it->second.get();
  auto pred = [&] { return r->done; };
  if (timeout_s < 0) {
    done_cv_.wait(lk, pred);
  } else if (!done_cv_.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
    return false;
  }
  out = *r;
  req_.erase(it);
  return true;
}

size_t Server::lane_bytes(int lattice) {
  std::lock_guard<std::mutex> lk(mu_);
  CRK_REQUIRE(lattice >= 0 && lattice < int(lat_.size()), "unknown lattice id");
  return lat_[lattice]->lane_bytes;
}

ServerStats Server::stats() {
  std::lock_guard<std::mutex> lk(mu_);
  return st_;
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  // Lanes drain their lattice's queue before they end; a lattice left with
  // queued requests and no lane gets one as soon as memory frees up.
  for (;;) {
    std::vector<Lane*> lanes;
    {
      std::lock_guard<std::mutex> lk(mu_);
      lanes = all_lanes_;
    }
    bool all_exited = true;
    for (Lane* l : lanes) {
      if (l->th.joinable()) l->th.join();
    }
    std::lock_guard<std::mutex> lk(mu_);
    for (Lane* l : all_lanes_) all_exited &= l->exited;
    bool pending = false;
    for (auto& e : lat_) pending |= !e->pending.empty();
    if (all_exited && all_lanes_.size() == lanes.size() && !pending) break;
    if (all_exited && all_lanes_.size() == lanes.size() && pending) {
      // nothing can run them any more (no lane fits): fail them
      for (size_t i = 0; i < lat_.size(); ++i) fail_pending_locked(int(i), CRK_ENOMEM, "server stopped");
      break;
    }
  }
  for (Lane* l : all_lanes_) delete l;
  for (auto& e : lat_) mg_destroy(e->H);
}

// ------------------------------------------------------------------ lane thread

void lane_main(Server* s, Lane* lane) {
  // The entry pointer was stored under the lock when the lane opened: lat_
  // itself may grow (and reallocate) while this thread runs.
  LatticeEntry& L = *lane->entry;
  Hierarchy* H = L.H;
  const int cap = s->p_.slots_per_lane;
  const int64_t per = 12 * H->V(0);  // complex entries per RHS
  hipStream_t st = nullptr;
  std::unique_ptr<Workspace> ws;
  std::unique_ptr<OuterSolver> os;
  DevBuf stage;
  std::vector<Request*> owner(cap, nullptr);
  std::vector<int> owner_rhs(cap, -1);
  auto fail_lane = [&](int code, const std::string& msg) {
    std::lock_guard<std::mutex> lk(s->mu_);
    for (int q = 0; q < cap; ++q) {
      Request* r = owner[q];
      if (r && !r->done) {
        r->status = code;
        r->error = msg;
        s->finish_locked(r);
      }
      owner[q] = nullptr;
    }
    s->close_lane_locked(lane);
    if (L.lanes.empty()) s->fail_pending_locked(lane->lattice, code, msg);
    lane->dead = true;
    lane->exited = true;
    s->open_lanes_locked();
    s->cv_.notify_all();
  };
  try {
    CRK_HIP(hipSetDevice(s->device_));
    CRK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    ws = make_workspace(H, cap, s->p_.solve.form, s->p_.solve, st);
    stage.alloc(sizeof(double2) * size_t(per) * cap);
    os = std::make_unique<OuterSolver>(H, ws.get(), s->p_.solve, st);
  } catch (const Error& e) {
    fail_lane(e.code, e.what());
    if (st) (void)hipStreamDestroy(st);
    return;
  } catch (const std::exception& e) {
    fail_lane(CRK_EINTERNAL, e.what());
    if (st) (void)hipStreamDestroy(st);
    return;
  }
  double2* stg = stage.as<double2>();
  bool closing = false;
  for (;;) {
    std::vector<std::pair<Request*, int>> admit;
    {
      std::unique_lock<std::mutex> lk(s->mu_);
      lane->ready = true;
      for (;;) {
        int fs = os->free_slots();
        const bool busy = os->running() > 0;
        while (!L.pending.empty()) {
          Request* r = L.pending.front();
          if (r->nrhs > fs) break;  // FIFO: the head waits for room
          L.pending.pop_front();
          r->lane = lane->id;
          r->t_admit = s->now();
          r->joined = busy;
          if (busy) s->st_.joins++;
          for (int i = 0; i < r->nrhs; ++i) admit.emplace_back(r, i);
          r->started = r->nrhs;
          fs -= r->nrhs;
        }
        lane->free_slots = fs;
        if (!admit.empty() || busy) break;
        // idle
        const double t = s->now();
        if (lane->idle_since < 0) lane->idle_since = t;
        if (s->stop_ && L.pending.empty()) { closing = true; break; }
        bool starving = false;
        for (auto& e : s->lat_)
          if (e.get() != &L && !e->pending.empty() && e->lanes.empty()) starving = true;
        const bool may_close = L.lanes.size() > 1 || starving;
        if (may_close && t - lane->idle_since >= 1e-3 * s->p_.idle_ms) { closing = true; break; }
        s->cv_.wait_for(lk, std::chrono::milliseconds(std::max(1, std::min(s->p_.idle_ms, 50))));
      }
      lane->idle_since = -1;
      if (closing) {
        s->close_lane_locked(lane);
        break;
      }
    }
    try {
      for (auto& [r, i] : admit) {
        const int q = os->first_free();
        CRK_REQUIRE(q >= 0, "no free slot for an admitted right-hand side");
        CRK_HIP(hipMemcpyAsync(stg + per * q, r->b + 2 * per * i, sizeof(double2) * size_t(per),
                               hipMemcpyHostToDevice, st));
        os->admit(q, 1, stg + per * q);
        owner[q] = r;
        owner_rhs[q] = i;
      }
      if (os->running() > 0) os->step();
      std::vector<int> fin;
      bool stopped = false;
      for (int q = 0; q < cap; ++q) {
        if (!owner[q] || os->state(q) == kSlotRunning) continue;
        fin.push_back(q);
        stopped |= os->state(q) == kSlotStopped;
      }
      if (fin.empty()) continue;
      if (stopped) os->refresh_residuals();
      std::vector<std::vector<std::vector<int>>> li(fin.size());
      for (size_t f = 0; f < fin.size(); ++f) {
        const int q = fin[f];
        os->export_x(q, 1, stg + per * q);
        CRK_HIP(hipMemcpyAsync(owner[q]->x + 2 * per * owner_rhs[q], stg + per * q, sizeof(double2) * size_t(per),
                               hipMemcpyDeviceToHost, st));
        os->level_iters(q, 1, li[f]);  // synchronises the stream
      }
      {
        std::lock_guard<std::mutex> lk(s->mu_);
        for (size_t f = 0; f < fin.size(); ++f) {
          const int q = fin[f];
          Request* r = owner[q];
          r->iters = std::max(r->iters, os->iters(q));
          for (int l = 1; l < CRK_MAX_LEVELS; ++l) r->level_iters[l] = std::max(r->level_iters[l], li[f][l][0]);
          r->level_iters[0] = r->iters;
          r->resid = std::max(r->resid, os->true_rel(q));
          if (os->state(q) == kSlotStopped && r->status == CRK_OK) {
            r->status = CRK_ENOCONV;
            r->error = "right-hand side did not converge within max_iter";
          }
          if (++r->finished == r->nrhs) s->finish_locked(r);
        }
      }
      for (int q : fin) {
        os->release(q);
        owner[q] = nullptr;
        owner_rhs[q] = -1;
      }
      {
        std::lock_guard<std::mutex> lk(s->mu_);
        lane->free_slots = os->free_slots();
        s->open_lanes_locked();
      }
    } catch (const Error& e) {
      fail_lane(e.code, e.what());
      break;
    } catch (const std::exception& e) {
      fail_lane(CRK_EINTERNAL, e.what());
      break;
    }
  }
  os.reset();
  ws.reset();
  stage.release();
  if (st) (void)hipStreamDestroy(st);
  std::lock_guard<std::mutex> lk(s->mu_);
  lane->exited = true;
  s->open_lanes_locked();
  s->cv_.notify_all();
}

}  // namespace crk
