// capi.h -- what the files of the C boundary share: the handle types behind
// include/ppstat.h's opaque structs and the exception-to-status guard.
#pragma once

#include "../../include/ppstat.h"

#include <new>

#include "server.h"

struct ppst_context {
  std::unique_ptr<ppst::Context> cx;
};
struct ppst_secret_key {
  std::unique_ptr<ppst::SecretKey> k;
};
struct ppst_public_key {
  std::unique_ptr<ppst::PublicKey> k;
};
struct ppst_eval_keys {
  ppst::EvalKeys e;
};
struct ppst_plaintext {
  ppst::PtPtr p;
};
struct ppst_ciphertext {
  ppst::CtPtr c;
};
struct ppst_server {
  std::unique_ptr<ppst::Server> s;
};
struct ppst_graph {
  std::unique_ptr<ppst::Graph> g;
};
namespace ppst {
struct Bootstrapper;
}
struct ppst_boot {
  std::unique_ptr<ppst::Bootstrapper> b;
  ~ppst_boot();
};

namespace ppst {

// the calling thread's last failure message (ppst_last_error)
std::string& last_error();

// runs f, turning a thrown Error into its status code and message
template <class F>
int guard(F&& f) {
  try {
    f();
    return PPST_OK;
  } catch (const Error& e) {
    last_error() = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    last_error() = "host allocation failed";
    return PPST_ENOMEM;
  } catch (const std::exception& e) {
    last_error() = e.what();
    return PPST_EINVAL;
  }
}

#define NEED(p)                                                   \
  do {                                                            \
    if (!(p)) PPST_THROW(ST_EINVAL, "null argument: " #p);          \
  } while (0)

inline ppst_ciphertext* wrap(CtPtr c) { return new ppst_ciphertext{std::move(c)}; }

// calls that wait for the device or move data to or from the host cannot be
// recorded into a graph
#define NOT_RECORDING(ctx)                                                       \
  do {                                                                           \
    if ((ctx)->cx->recording)                                                    \
      PPST_THROW(ST_EINVAL, "not allowed while a graph recording is open");      \
  } while (0)

// the library's parameter specification of a ppst_params
ParamSpec spec_from(const ppst_params& p);

// Device-side scratch of ppst_mul_noalloc: sets up the current device's
// array (once per device; context creation calls it) and returns its
// address, or throws when the runtime could not resolve it.
u64* noalloc_scratch();
size_t noalloc_scratch_bytes();

}  // namespace ppst
