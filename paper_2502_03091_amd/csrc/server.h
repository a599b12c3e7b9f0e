// Continuously batched solve server.
//
// Hierarchies (gauge field, P, coarse operators) stay resident on the device.
// Every registered lattice owns a FIFO of solve requests and up to max_lanes
// *lanes*: a lane is one outer MG-GCR solver with a fixed number of RHS slots,
// its own buffers, HIP stream and host thread.  Between two outer iterations a
// lane retires the slots whose RHS have finished (true residual verified,
// result copied out) and admits queued requests into free slots while the
// other RHS keep iterating.  A new lane is opened when queued RHS exceed the
// free slots of a lattice's lanes and its buffers fit in the HBM budget; idle
// lanes beyond the first close again and give their memory back.  Lanes of
// different lattices (and several lanes of one lattice) run concurrently on
// their own streams.
#pragma once

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "solver.h"

namespace crk {

struct Request {
  uint64_t id = 0;
  int lattice = 0;
  const double* b = nullptr;  // caller-owned complex128 [nrhs][V][12]
  double* x = nullptr;
  int nrhs = 0;
  int started = 0, finished = 0;  // RHS admitted / done
  int lane = -1;
  bool joined = false;            // admitted while the lane had RHS in flight
  bool done = false;
  int status = CRK_OK;
  std::string error;
  int iters = 0;
  int level_iters[CRK_MAX_LEVELS] = {0, 0, 0};
  double resid = 0;
  double t_submit = 0, t_admit = -1, t_done = 0;
};

class Server;
struct Lane;
void lane_main(Server* s, Lane* lane);

struct LatticeEntry;

struct Lane {
  Server* srv = nullptr;
  LatticeEntry* entry = nullptr;  // set under the server lock when the lane opens; the entry never moves
  int lattice = 0, id = 0;
  bool ready = false, dead = false, exited = false;
  int free_slots = 0;      // mirrored under the server lock
  double idle_since = 0;
  size_t bytes = 0;
  std::thread th;
};

struct LatticeEntry {
  Hierarchy* H = nullptr;
  size_t lane_bytes = 0;
  std::deque<Request*> pending;
  std::vector<Lane*> lanes;
  int next_lane_id = 0;
};

struct ServerStats {
  int64_t submitted = 0, completed = 0, failed = 0, joins = 0;
  int64_t lanes_opened = 0, lanes_closed = 0, max_concurrent_lanes = 0;
  int64_t bytes_in_use = 0, peak_bytes = 0;
};

class Server {
 public:
  Server(const crk_server_params& p);
  ~Server();
  int add(Hierarchy* H);
  uint64_t submit(int lattice, const double* b, double* x, int nrhs);
  // Waits for a request; false on timeout.  Fills the result and forgets the request.
  bool wait(uint64_t id, double timeout_s, Request& out);
  ServerStats stats();
  double now() const;
  size_t budget() const { return budget_; }
  size_t lane_bytes(int lattice);

 private:
  friend void lane_main(Server* s, Lane* lane);
  crk_server_params p_;
  int device_ = 0;
  std::chrono::steady_clock::time_point t0_;
  std::mutex mu_;
  std::condition_variable cv_;       // lanes: work arrived / stop
  std::condition_variable done_cv_;  // waiters: a request finished
  bool stop_ = false;
  std::vector<std::unique_ptr<LatticeEntry>> lat_;
  std::vector<Lane*> all_lanes_;     // every lane ever opened (joined and freed at destruction)
  std::map<uint64_t, std::unique_ptr<Request>> req_;
  uint64_t next_id_ = 1;
  size_t budget_ = 0;
  ServerStats st_;
  int open_lanes_ = 0;

  void open_lanes_locked();
  void finish_locked(Request* r);
  void fail_pending_locked(int lattice, int code, const std::string& msg);
  void close_lane_locked(Lane* ln);
};

}  // namespace crk
