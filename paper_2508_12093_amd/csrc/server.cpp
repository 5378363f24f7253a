// server.cpp -- encrypted-statistics serving: admission by free device memory
// and in-flight slots, one HIP stream per worker so that admitted queries
// overlap on the GPU, columns and evaluation keys resident in HBM.
#include "server.h"

#include <chrono>

namespace ppst {

double now_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

Server::Server(Context& base, std::shared_ptr<const EvalKeys> evk, size_t budget, int slots)
    : sh_(base.sh), evk_(std::move(evk)), budget_(budget) {
  if (slots < 1 || slots > 16) PPST_THROW(ST_EINVAL, "server slots must be in 1..16");
  // the evaluation keys may still be being generated on the caller's stream;
  // the workers read them from their own streams
  HIP_CHECK(hipDeviceSynchronize());
  base_ = make_context(sh_, nullptr);
  for (int i = 0; i < slots; ++i) workers_cx_.push_back(make_context(sh_, nullptr));
  for (int i = 0; i < slots; ++i) threads_.emplace_back([this, i] { worker(i); });
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
  }
  cv_work_.notify_all();
  for (auto& t : threads_) t.join();
  for (auto& c : workers_cx_) destroy_context(c.get());
  states_.clear();
  columns_.clear();
  destroy_context(base_.get());
}

u64 Server::register_column(const std::vector<const Ciphertext*>& cts, size_t nrows) {
  if (cts.empty()) PPST_THROW(ST_EINVAL, "empty column");
  size_t need = (nrows + sh_->P.slots() - 1) / sh_->P.slots();
  if (nrows == 0 || need != cts.size()) PPST_THROW(ST_EINVAL, "row count does not match the column");
  Column col;
  col.nrows = nrows;
  // the ciphertexts may still be in flight on the stream of whichever context
  // produced them (an encryption is asynchronous): let every stream drain
  // before copying, registration is not on the query path
  HIP_CHECK(hipDeviceSynchronize());
  for (auto* c : cts) col.cts.push_back(copy_ct(*base_, *c));
  HIP_CHECK(hipStreamSynchronize(base_->stream));
  std::lock_guard<std::mutex> g(mu_);
  u64 id = next_col_++;
  columns_[id] = std::move(col);
  return id;
}

// Device memory a query may hold at its peak: the key-switching scratch of one
// product at the column's level (input copy, beta extended digits, two
// extended accumulators, the ModDown conversion) plus the live ciphertexts of
// the circuit (a fixed allowance of 24, and 4 per column ciphertext).
size_t Server::estimate_bytes(const Query& q) const {
  const Params& P = sh_->P;
  auto it = columns_.find(q.col_x);
  if (it == columns_.end()) PPST_THROW(ST_EINVAL, "unknown column");
  const int level = it->second.cts[0]->level;
  const size_t nl = level + 1, ne = nl + P.K, beta = P.beta(level);
  size_t limbs = nl + beta * ne + 2 * ne + 2 * nl;
  size_t cts = 24 + 4 * it->second.cts.size();
  if (q.kind == 4) cts += 4 * it->second.cts.size();
  limbs += cts * 2 * nl;
  return limbs * (size_t)P.N * 8;
}

u64 Server::submit(const Query& q) {
  std::lock_guard<std::mutex> g(mu_);
  if (!columns_.count(q.col_x) || (q.kind == 4 && !columns_.count(q.col_y)))
    PPST_THROW(ST_EINVAL, "unknown column handle");
  if (q.kind < 0 || q.kind > 6) PPST_THROW(ST_EINVAL, "unknown query kind");
  auto st = std::make_shared<QueryState>();
  st->q = q;
  st->ticket = next_ticket_++;
  st->bytes = estimate_bytes(q);
  if (st->bytes > budget_)
    PPST_THROW(ST_ENOMEM, "query needs " + std::to_string(st->bytes) + " bytes, budget is " +
                            std::to_string(budget_));
  st->t_submit = now_seconds();
  states_[st->ticket] = st;
  pending_.push_back(st->ticket);
  cv_work_.notify_all();
  return st->ticket;
}

std::vector<CtPtr> Server::run(Context& cx, const QueryState& st) {
  const Query& q = st.q;
  const Column& X = st.X;
  switch (q.kind) {
    case 0: return {stat_mean(cx, *evk_, X.cts, X.nrows, q.B)};
    case 1: return {stat_variance(cx, *evk_, X.cts, X.nrows, q.B)};
    case 2: return stat_zscore(cx, *evk_, X.cts, X.nrows, q.B, q.cfg);
    case 3: return {stat_cv(cx, *evk_, X.cts, X.nrows, q.B, q.B2, q.cfg, q.sign_k)};
    case 4: {
      const Column& Y = st.Y;
      if (Y.nrows != X.nrows) PPST_THROW(ST_EINVAL, "columns differ in row count");
      return {stat_pearson(cx, *evk_, X.cts, Y.cts, X.nrows, q.B, q.B2, q.cfg)};
    }
    case 5: return {stat_skewness(cx, *evk_, X.cts, X.nrows, q.B, q.cfg)};
    case 6: return {stat_kurtosis(cx, *evk_, X.cts, X.nrows, q.B, q.cfg, false)};
  }
  PPST_THROW(ST_EINVAL, "unknown query kind");
}

void Server::worker(int idx) {
  Context& cx = *workers_cx_[idx];
  HIP_CHECK(hipSetDevice(sh_->device));
  for (;;) {
    std::shared_ptr<QueryState> st;
    {
      std::unique_lock<std::mutex> g(mu_);
      // admit the oldest pending query once its memory fits
      cv_work_.wait(g, [&] {
        return stop_ || (!pending_.empty() && reserved_ + states_[pending_.front()]->bytes <= budget_);
      });
      if (stop_) return;
      st = states_[pending_.front()];
      pending_.pop_front();
      st->X = columns_[st->q.col_x];
      if (st->q.kind == 4) st->Y = columns_[st->q.col_y];
      reserved_ += st->bytes;
      st->t_admit = now_seconds();
    }
    try {
      st->results = run(cx, *st);
      HIP_CHECK(hipStreamSynchronize(cx.stream));
      st->status = ST_OK;
    } catch (const Error& e) {
      (void)hipStreamSynchronize(cx.stream);
      st->status = e.code;
      st->error = e.what();
      st->results.clear();
    } catch (const std::exception& e) {
      (void)hipStreamSynchronize(cx.stream);
      st->status = ST_EINVAL;
      st->error = e.what();
      st->results.clear();
    }
    {
      std::lock_guard<std::mutex> g(mu_);
      st->t_done = now_seconds();
      st->done = true;
      reserved_ -= st->bytes;
    }
    cv_done_.notify_all();
    cv_work_.notify_all();
  }
}

bool Server::poll(u64 ticket) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = states_.find(ticket);
  if (it == states_.end()) PPST_THROW(ST_EINVAL, "unknown ticket");
  return it->second->done;
}

size_t Server::output_count(u64 ticket) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = states_.find(ticket);
  if (it == states_.end()) PPST_THROW(ST_EINVAL, "unknown ticket");
  const Query& q = it->second->q;
  if (q.kind != 2) return 1;
  auto c = columns_.find(q.col_x);
  return c == columns_.end() ? 1 : c->second.cts.size();
}

int Server::wait(u64 ticket, std::vector<CtPtr>* out, QueryState* stats) {
  std::unique_lock<std::mutex> g(mu_);
  auto it = states_.find(ticket);
  if (it == states_.end()) PPST_THROW(ST_EINVAL, "unknown ticket");
  auto st = it->second;
  cv_done_.wait(g, [&] { return st->done; });
  states_.erase(ticket);
  if (stats) {
    stats->t_submit = st->t_submit;
    stats->t_admit = st->t_admit;
    stats->t_done = st->t_done;
    stats->bytes = st->bytes;
    stats->status = st->status;
    stats->error = st->error;
  }
  if (out) *out = st->results;
  return st->status;
}

}  // namespace ppst
