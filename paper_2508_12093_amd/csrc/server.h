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
  bool done = false;
};

class Server {
 public:
  Server(Context& base, std::shared_ptr<const EvalKeys> evk, size_t budget, int slots);
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

 private:
  void worker(int idx);
  std::vector<CtPtr> run(Context& cx, const QueryState& st);

  std::shared_ptr<Shared> sh_;
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
