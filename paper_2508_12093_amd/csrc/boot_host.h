// boot_host.h -- host-side constants of CKKS bootstrapping's linear transforms
// (plain C++; built without the HIP headers, in binary128 arithmetic).
#pragma once

#include <cstdint>
#include <vector>

namespace ppst {

// One level of CoeffToSlot (inverse = 1) or SlotToCoeff (inverse = 0): the
// special-FFT butterfly layers len = 2^lo .. 2^hi merged into one sparse
// matrix, evaluated by baby steps and giant steps over offsets
// u (m0 + b j + i), 0 <= i < b, 0 <= j < G.
struct BootGroup {
  int inverse = 0, lo = 0, hi = 0, level = 0, ckind = 0, u = 0, m0 = 0, b = 0, G = 0;
};

// The numbers a group's plaintext factor is formed from: the plaintext scale
// Delta_{l-1} q_l / Delta_l that brings a ciphertext at Delta_l to
// Delta_{l-1} through one rescale, times the transform's constant c
// (ckind 0: 1; 1: Delta_L / (2 K q_0); 2: (q_0 / (2 pi Delta_0))^(1/nsplit)).
struct BootFactor {
  double scale_out = 0, scale_in = 0;
  uint64_t q_l = 0;
  double scale_top = 0;
  uint64_t q0 = 0;
  double scale0 = 0;
  int K = 0, nsplit = 1;
};

// Integer coefficients of every cell's plaintext, out [G b][N] (row j b + i):
// the diagonal of offset u (m0 + b j + i) mod n, rotated by -u (m0 + b j) and
// encoded (coefficient k = round_half_away(S (2/N) Re sum_s v_s xi_s^(-k)),
// S the factor) in binary128; used[j b + i] = 0 where the group has no such
// diagonal.  Throws std::runtime_error when a diagonal falls outside the grid
// or a coefficient leaves int64.  Uses up to `threads` host threads.
void boot_group_coeffs(int logN, const BootGroup& g, const BootFactor& f, int64_t* out,
                       uint8_t* used, int threads);

// The group's factor in double precision (for reporting)
double boot_group_factor(const BootGroup& g, const BootFactor& f);

}  // namespace ppst
