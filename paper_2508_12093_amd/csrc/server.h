// server.h -- request loop for encrypted-statistics queries over resident columns.
#pragma once

#include <condition_variable>
#include <deque>
#include <thread>

#include "stats.h"

namespace ppst {

struct Query {
  int kind = 0;
  u64 col_x = 0, col_y = 0;
  double B = 1.0, B2 = 1.0;
  InvSqrtCfg cfg;
  int sign_k = 2;
};

// Merges the rotate-and-sums of queries in flight on different workers into
// shared launches.  The first worker to reach one at a level waits a short
// window for others at the same level (until max_lanes lanes are pending,
// every busy worker is waiting, or the window ends), then runs all their
// lanes as one rotsum_batch on its own stream: after the requesters' events,
// into result ciphertexts each requester allocated on its own pool, followed
// by an event every requester's stream waits on before its next launch.  The
// batched form is bit for bit the one-lane form, so results do not depend on
// what was merged.
class RotSumMerger : public RotSumRouter {
 public:
  RotSumMerger(int max_lanes, double window_s) : max_lanes_(max_lanes), window_s_(window_s) {}
  std::vector<CtPtr> rotsum(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& lanes) override;
  void busy(int delta);
  // launches run, lanes served, launches that carried more than one query's lanes
  void counters(u64* launches, u64* lanes, u64* merged) const;

 private:
  struct Request;
  int max_lanes_;
  double window_s_;
  mutable std::mutex mu_;
  std::condition_variable cv_;
  std::map<int, std::vector<std::shared_ptr<Request>>> queue_;   // by level
  int busy_ = 0, waiting_ = 0;
  u64 launches_ = 0, lanes_ = 0, merged_ = 0;
};

struct Column {
  std::vector<CtPtr> cts;
  size_t nrows = 0;
};

struct QueryState {
  Query q;
  Column X, Y;                 // the query's columns, captured at admission
  u64 ticket = 0;
  size_t bytes = 0;
  int status = 0;
  std::string error;
  std::vector<CtPtr> results;  // ZNorm: one per column ciphertext; else one
  double t_submit = 0, t_admit = 0, t_done = 0;
  size_t peak = 0;             // device bytes the query's worker pool took at most
  bool done = false;
};

class Server {
 public:
  // budget 0: the device's free memory at creation, less a margin.  merge:
  // route the circuits' rotate-and-sums through a RotSumMerger.
  Server(Context& base, std::shared_ptr<const EvalKeys> evk, size_t budget, int slots,
         bool merge = true);
  ~Server();
  u64 register_column(const std::vector<const Ciphertext*>& cts, size_t nrows);
  u64 submit(const Query& q);
  // blocks; returns the query's status and moves the results out
  int wait(u64 ticket, std::vector<CtPtr>* out, QueryState* stats);
  // number of result ciphertexts the query produces (ZNorm: its column's
  // ciphertext count; otherwise 1)
  size_t output_count(u64 ticket);
  // whether the query has finished (its result stays until wait() collects it)
  bool poll(u64 ticket);
  size_t estimate_bytes(const Query& q) const;
  size_t budget() const { return budget_; }
  void merge_counters(u64* launches, u64* lanes, u64* merged) const;

 private:
  void worker(int idx);
  std::vector<CtPtr> run(Context& cx, const QueryState& st);

  std::shared_ptr<Shared> sh_;
  std::unique_ptr<RotSumMerger> merger_;
  std::unique_ptr<Context> base_;
  std::shared_ptr<const EvalKeys> evk_;
  size_t budget_;
  std::vector<std::unique_ptr<Context>> workers_cx_;
  std::vector<std::thread> threads_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<u64> pending_;
  std::map<u64, std::shared_ptr<QueryState>> states_;
  std::map<u64, Column> columns_;
  size_t reserved_ = 0;
  u64 next_ticket_ = 1, next_col_ = 1;
  bool stop_ = false;
};

double now_seconds();

}  // namespace ppst
