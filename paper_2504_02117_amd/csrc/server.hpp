// Serving loop state (server.cpp).
#pragma once

#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "serve.hpp"

struct bkts_server_s {
  struct Pending {
    bkts_request req{};
    uint64_t ticket = 0;
    double t_submit = 0.0;
    size_t footprint = 0;
  };
  struct OpDel {
    void operator()(bkts_op o) const { delete o; }
  };
  struct TcDel {
    void operator()(bkts_tc t) const { delete t; }
  };
  struct Job {
    enum State { RESID, INIT, CG, FINISHING };
    Pending p;
    double t_admit = 0.0;
    std::unique_ptr<bkts_op_s, OpDel> op;
    std::unique_ptr<bkts_tc_s, TcDel> tc;
    int64_t N = 0;
    int k = 1, kp = 1, nb0 = 1;
    double beta = 1.0, rhs0 = 0.0, rel = 0.0;
    bkts::DevBuf Y, R64, f32, dinv, B0, part, small;
    double *sc = nullptr, *sp = nullptr, *mats = nullptr, *nrm64 = nullptr, *nrm0 = nullptr;
    bkts::GJob g{};
    State state = RESID;
    bool pending_apply = false;
    int outer = 0, inner_it = 0, krylov = 0, final_status = BKTS_OK;
  };

  // A worker lane for mode-1 (pipelined) requests: its own thread, context and stream.
  struct Lane {
    bkts_ctx ctx = nullptr;
    std::thread th;
    bool busy = false;  // a request is assigned (guarded by mu)
    Pending p;
  };
  static constexpr int kLanes = 16;  // at most; a server has min(kLanes, max_slots)
  int nlanes = 0;

  bkts_ctx ctx = nullptr;  // the server's own context and stream
  size_t budget;
  int max_slots;
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<Pending> queue;
  std::deque<bkts_result> done;
  bool stop = false, fatal = false;
  std::string fatal_msg;
  uint64_t next_ticket = 0;
  size_t in_use = 0, peak = 0;
  int n_active = 0, max_active = 0;
  long rounds = 0, grouped_launches = 0;

  // worker-only state
  std::vector<std::unique_ptr<Job>> jobs;  // one per slot
  Lane lanes[kLanes];
  bkts::DevBuf status_dev, table_dev;
  double* status_host = nullptr;
  void* table_host = nullptr;
  size_t table_bytes = 0;
  std::thread worker;

  bkts_server_s(int device, size_t budget, int max_slots);
  ~bkts_server_s();
  static size_t footprint(const bkts_request& r);
  static size_t footprint_pipelined(const bkts_request& r);
  double now() const;
  uint64_t submit(const bkts_request& r);
  int poll(bkts_result* out, int max);
  int wait(int n, double timeout_s);
  bkts_server_stats stats();

 private:
  void run();
  void lane_run(int l);
  bkts_result lane_solve(Lane& L, const Pending& p);
  int n_active_now();
  void setup(int slot, const Pending& p);
  void round();
  void finish(int slot, int status);
};
