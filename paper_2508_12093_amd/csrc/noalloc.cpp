// noalloc.cpp -- ppst_mul_noalloc: HMult+relin+rescale into caller memory
// without any device allocation, its key-switching intermediates in one
// file-scope device array per GPU.
#include <mutex>

#include "capi.h"

using namespace ppst;

namespace {

// Enough for a product at level 24 of N = 2^16 with 7 special primes and
// three digits (283 limbs of 512 KiB); larger shapes are refused.
constexpr size_t kScratchBytes = (size_t)144 << 20;

// Every GPU the library runs on holds its own copy until the process ends.
// Host code never passes this name to a kernel or a copy (on the host it is
// only a stand-in for the symbol): it uses the address resolved below.
static __device__ __align__(256) u64 scratch[kScratchBytes / sizeof(u64)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
u64* g_ptr[kMaxDevices] = {};
std::string g_fail[kMaxDevices];

}  // namespace

namespace ppst {

size_t noalloc_scratch_bytes() { return kScratchBytes; }

u64* noalloc_scratch() {
  int dev = -1;
  HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) PPST_THROW(ST_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> g(g_mu);
  if (g_ptr[dev]) return g_ptr[dev];
  if (!g_fail[dev].empty()) PPST_THROW(ST_EDEVICE, g_fail[dev]);
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    g_fail[dev] = std::string("hipGetSymbolAddress of the no-allocation scratch failed: ") +
                  hipGetErrorString(e);
    PPST_THROW(ST_EDEVICE, g_fail[dev]);
  }
  g_ptr[dev] = (u64*)p;
  return g_ptr[dev];
}

}  // namespace ppst

extern "C" int ppst_mul_noalloc(ppst_context* ctx, const ppst_eval_keys* evk, const uint64_t* a,
                                const uint64_t* b, int32_t level, uint64_t* out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(a); NEED(b); NEED(out);
    Context& cx = *ctx->cx;
    const Params& P = cx.P();
    if (level < 1 || level > P.L)
      PPST_THROW(ST_ELEVEL, "a product needs a level in 1.." + std::to_string(P.L));
    const size_t need = mul_scratch_words(P, level) * sizeof(u64);
    if (need > kScratchBytes)
      PPST_THROW(ST_EINVAL, "a product at level " + std::to_string(level) + " needs " +
                             std::to_string(need) + " bytes of scratch; the no-allocation form "
                             "holds " + std::to_string(kScratchBytes));
    const size_t in_words = 2 * ((size_t)level + 1) * P.N, out_words = 2 * (size_t)level * P.N;
    if ((out < a + in_words && a < out + out_words) || (out < b + in_words && b < out + out_words))
      PPST_THROW(ST_EINVAL, "the output overlaps an operand");
    mul_into(cx, evk->e, a, b, level, out, noalloc_scratch());
  });
}
