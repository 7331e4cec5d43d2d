// Linear inequalities G x >= h (Section 3.4): the slack form of the
// program and its kernel basis [B; G B] (the corollary of that section).
// Host code; the lifted program then runs through the ordinary entry points
// (the descent kernels see a basis with n + m' rows).
#include <cstring>
#include <vector>

#include "graver_internal.h"

using namespace graver;

namespace {

bool add_ok(__int128 v) { return v > -((__int128)1 << 62) && v < ((__int128)1 << 62); }

}  // namespace

extern "C" graver_status graver_lift_inequalities(int32_t m, int32_t n, const int64_t* A, const int64_t* b,
                                                  const int64_t* l, const int64_t* u, int32_t mi,
                                                  const int64_t* G, const int64_t* h, int32_t d,
                                                  const int64_t* B, int64_t* A_out, int64_t* b_out,
                                                  int64_t* l_out, int64_t* u_out, int64_t* Bt_out) {
  if (m < 0 || n < 1 || mi < 1 || d < 0) return set_error(GRAVER_E_INVALID, "need m >= 0, n >= 1, m' >= 1");
  if ((m > 0 && (!A || !b)) || !l || !u || !G || !h || !A_out || !b_out || !l_out || !u_out)
    return set_error(GRAVER_E_INVALID, "NULL argument");
  if (B && (d < 1 || !Bt_out)) return set_error(GRAVER_E_INVALID, "B needs d >= 1 and Bt_out");
  const int n2 = n + mi, m2 = m + mi;
  // slack bounds first (error before any output is written)
  std::vector<int64_t> smax(mi);
  for (int i = 0; i < mi; ++i) {
    __int128 t = 0;
    for (int j = 0; j < n; ++j) {
      const __int128 g = G[(size_t)i * n + j];
      const __int128 a = g * l[j], c = g * u[j];
      t += a > c ? a : c;
      if (!add_ok(t)) return set_error(GRAVER_E_OVERFLOW, "slack bound overflows int64");
    }
    t -= h[i];
    if (!add_ok(t)) return set_error(GRAVER_E_OVERFLOW, "slack bound overflows int64");
    if (t < 0) return set_error(GRAVER_E_INVALID, "an inequality cannot hold anywhere in the box");
    smax[i] = (int64_t)t;
  }
  std::vector<int64_t> GB;
  if (B) {
    GB.assign((size_t)mi * d, 0);
    for (int i = 0; i < mi; ++i)
      for (int c = 0; c < d; ++c) {
        __int128 t = 0;
        for (int j = 0; j < n; ++j) {
          t += (__int128)G[(size_t)i * n + j] * B[(size_t)j * d + c];
          if (!add_ok(t)) return set_error(GRAVER_E_OVERFLOW, "G B overflows int64");
        }
        GB[(size_t)i * d + c] = (int64_t)t;
      }
  }
  std::memset(A_out, 0, sizeof(int64_t) * (size_t)m2 * n2);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) A_out[(size_t)i * n2 + j] = A[(size_t)i * n + j];
  for (int i = 0; i < mi; ++i) {
    for (int j = 0; j < n; ++j) A_out[(size_t)(m + i) * n2 + j] = G[(size_t)i * n + j];
    A_out[(size_t)(m + i) * n2 + n + i] = -1;
  }
  for (int i = 0; i < m; ++i) b_out[i] = b[i];
  for (int i = 0; i < mi; ++i) b_out[m + i] = h[i];
  for (int j = 0; j < n; ++j) {
    l_out[j] = l[j];
    u_out[j] = u[j];
  }
  for (int i = 0; i < mi; ++i) {
    l_out[n + i] = 0;
    u_out[n + i] = smax[i];
  }
  if (B) {
    for (int j = 0; j < n; ++j)
      for (int c = 0; c < d; ++c) Bt_out[(size_t)j * d + c] = B[(size_t)j * d + c];
    for (int i = 0; i < mi; ++i)
      for (int c = 0; c < d; ++c) Bt_out[(size_t)(n + i) * d + c] = GB[(size_t)i * d + c];
  }
  return GRAVER_OK;
}
