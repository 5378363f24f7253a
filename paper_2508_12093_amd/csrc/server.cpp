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

// ----------------------------------------------------- merged rotate-and-sum
namespace {
struct Event {
  hipEvent_t e = nullptr;
  Event() { HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming)); }
  ~Event() { (void)hipEventDestroy(e); }
  Event(const Event&) = delete;
  Event& operator=(const Event&) = delete;
};
}  // namespace

struct RotSumMerger::Request {
  std::vector<CtPtr> lanes;     // the requester's inputs (its stream's results)
  std::vector<CtPtr> outs;      // results, allocated on the requester's pool
  std::shared_ptr<Event> ready; // the inputs are complete after this
  std::shared_ptr<Event> done;  // the results are complete after this
  bool finished = false;
  int status = ST_OK;
  std::string error;
};

void RotSumMerger::busy(int delta) {
  std::lock_guard<std::mutex> g(mu_);
  busy_ += delta;
  cv_.notify_all();
}

void RotSumMerger::counters(u64* launches, u64* lanes, u64* merged) const {
  std::lock_guard<std::mutex> g(mu_);
  *launches = launches_;
  *lanes = lanes_;
  *merged = merged_;
}

std::vector<CtPtr> RotSumMerger::rotsum(Context& cx, const EvalKeys& evk,
                                        const std::vector<CtPtr>& lanes) {
  if (lanes.empty()) return {};
  const int level = lanes[0]->level;
  for (const CtPtr& c : lanes)
    if (c->level != level || c->npoly != 2) return rotsum_batch(cx, evk, lanes);
  auto req = std::make_shared<Request>();
  req->lanes = lanes;
  for (const CtPtr& c : lanes) req->outs.push_back(new_ct(cx, level, c->scale));
  req->ready = std::make_shared<Event>();
  HIP_CHECK(hipEventRecord(req->ready->e, cx.stream));

  std::unique_lock<std::mutex> g(mu_);
  auto& q = queue_[level];
  q.push_back(req);
  ++waiting_;
  cv_.notify_all();
  if (q.size() == 1) {
    // leader: gather the lanes of other workers reaching a rotate-and-sum at
    // this level within the window
    auto pending = [&] {
      size_t n = 0;
      for (auto& r : queue_[level]) n += r->lanes.size();
      return n;
    };
    const auto until = std::chrono::steady_clock::now() +
                       std::chrono::microseconds((long)(window_s_ * 1e6));
    cv_.wait_until(g, until, [&] { return (int)pending() >= max_lanes_ || waiting_ >= busy_; });
    std::vector<std::shared_ptr<Request>> batch;
    std::swap(batch, queue_[level]);
    queue_.erase(level);
    waiting_ -= (int)batch.size();
    g.unlock();
    auto done = std::make_shared<Event>();
    int status = ST_OK;
    std::string error;
    try {
      std::vector<CtPtr> in, out;
      for (auto& r : batch) {
        HIP_CHECK(hipStreamWaitEvent(cx.stream, r->ready->e, 0));
        in.insert(in.end(), r->lanes.begin(), r->lanes.end());
        out.insert(out.end(), r->outs.begin(), r->outs.end());
      }
      rotsum_batch_into(cx, evk, in, out);
      HIP_CHECK(hipEventRecord(done->e, cx.stream));
    } catch (const Error& e) {
      status = e.code;
      error = e.what();
    } catch (const std::exception& e) {
      status = ST_EINVAL;
      error = e.what();
    }
    g.lock();
    ++launches_;
    if (batch.size() > 1) ++merged_;
    for (auto& r : batch) {
      lanes_ += r->lanes.size();
      r->done = done;
      r->status = status;
      r->error = error;
      r->finished = true;
    }
    cv_.notify_all();
  } else {
    cv_.wait(g, [&] { return req->finished; });
  }
  g.unlock();
  if (req->status != ST_OK) PPST_THROW(req->status, req->error);
  // nothing more runs on this stream before the merged launch has written
  // the results (and read the inputs, which this worker may then release)
  HIP_CHECK(hipStreamWaitEvent(cx.stream, req->done->e, 0));
  return req->outs;
}

// lanes one merged rotate-and-sum launch gathers (two key reads of the
// five-lane inner product) and how long its first worker waits for them
constexpr int kMergeLanes = 10;
constexpr double kMergeWindowS = 500e-6;

Server::Server(Context& base, std::shared_ptr<const EvalKeys> evk, size_t budget, int slots,
               bool merge)
    : sh_(base.sh), evk_(std::move(evk)), budget_(budget) {
  if (slots < 1 || slots > 16) PPST_THROW(ST_EINVAL, "server slots must be in 1..16");
  // the evaluation keys may still be being generated on the caller's stream;
  // the workers read them from their own streams
  HIP_CHECK(hipDeviceSynchronize());
  if (budget_ == 0) {
    // admission by the device's free memory: what is free now, less 2 GiB
    // for the tables' and keys' growth and the runtime
    size_t free_b = 0, total_b = 0;
    HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
    const size_t margin = (size_t)2 << 30;
    budget_ = free_b > margin ? free_b - margin : 0;
  }
  if (merge) merger_.reset(new RotSumMerger(kMergeLanes, kMergeWindowS));
  base_ = make_context(sh_, nullptr);
  for (int i = 0; i < slots; ++i) {
    workers_cx_.push_back(make_context(sh_, nullptr));
    workers_cx_.back()->router = merger_.get();
  }
  for (int i = 0; i < slots; ++i) threads_.emplace_back([this, i] { worker(i); });
}

void Server::merge_counters(u64* launches, u64* lanes, u64* merged) const {
  *launches = *lanes = *merged = 0;
  if (merger_) merger_->counters(launches, lanes, merged);
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
// extended accumulators, the ModDown conversion), the scratch of its widest
// rotate-and-sum (lanes x (coefficient copy, extended digits, accumulators);
// in a merged launch the leader holds every participant's lanes, which their
// own estimates cover), plus the live ciphertexts of the circuit (a fixed
// allowance of 24, and 4 per column ciphertext), all rounded as the pool
// rounds its blocks.
size_t Server::estimate_bytes(const Query& q) const {
  const Params& P = sh_->P;
  auto it = columns_.find(q.col_x);
  if (it == columns_.end()) PPST_THROW(ST_EINVAL, "unknown column");
  const int level = it->second.cts[0]->level;
  const size_t nl = level + 1, ne = nl + P.K, beta = P.beta(level);
  size_t limbs = nl + beta * ne + 2 * ne + 2 * nl;
  static const size_t kLanes[7] = {1, 1, 2, 2, 5, 2, 2};   // mean var z cv pcc skew kurt
  limbs += kLanes[q.kind < 0 || q.kind > 6 ? 4 : q.kind] * (nl + beta * ne + 2 * ne);
  size_t cts = 24 + 4 * it->second.cts.size();
  if (q.kind == 4) cts += 4 * it->second.cts.size();
  limbs += cts * 2 * nl;
  // the pool hands out blocks rounded up to its size classes, at most 25 %
  // above the request
  return limbs * (size_t)P.N * 8 / 4 * 5;
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
    cx.pool->reset_peak();
    const size_t base_use = cx.pool->in_use();
    if (merger_) merger_->busy(+1);
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
    if (merger_) merger_->busy(-1);
    {
      std::lock_guard<std::mutex> g(mu_);
      st->t_done = now_seconds();
      st->peak = cx.pool->peak() - base_use;
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
    stats->peak = st->peak;
    stats->status = st->status;
    stats->error = st->error;
  }
  if (out) *out = st->results;
  return st->status;
}

}  // namespace ppst
