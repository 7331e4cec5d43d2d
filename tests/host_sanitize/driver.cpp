// The host-only parts of the library -- the kernel basis (Lemma 3.1,
// Theorem 3.2, Appendix A, and the reduction-interleaved elimination) and
// the inequality lift (Section 3.4) -- built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  Reads
// instances from the file named by argv[1], writes results to argv[2]:
//   basis m n lll A(row-major)      ->  basis st d B(row-major) P(%.17g)
//   lift m n mi A b l u G h         ->  lift st A' b' l' u'
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "graver_internal.h"

namespace graver {
graver_status set_error(graver_status s, const std::string& msg) {
  std::fprintf(stderr, "library error %d: %s\n", (int)s, msg.c_str());
  return s;
}
graver_status hip_error(hipError_t, const char* what) { return set_error(GRAVER_E_DEVICE, what); }
}  // namespace graver

static std::vector<int64_t> read_vec(FILE* f, size_t k) {
  std::vector<int64_t> v(k);
  for (size_t i = 0; i < k; ++i)
    if (std::fscanf(f, "%ld", &v[i]) != 1) throw std::runtime_error("short input");
  return v;
}

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* in = std::fopen(argv[1], "r");
  FILE* out = std::fopen(argv[2], "w");
  if (!in || !out) return 2;
  char kind[16];
  while (std::fscanf(in, "%15s", kind) == 1) {
    if (std::string(kind) == "basis") {
      int m, n, lll;
      if (std::fscanf(in, "%d %d %d", &m, &n, &lll) != 3) return 2;
      std::vector<int64_t> A = read_vec(in, (size_t)m * n);
      std::vector<int64_t> B((size_t)n * n);
      std::vector<double> P((size_t)n * n);
      int32_t d = 0;
      graver_status st = graver::kernel_basis_host(m, n, A.data(), lll, B.data(), &d, P.data());
      std::fprintf(out, "basis %d %d", (int)st, d);
      if (st == GRAVER_OK) {
        for (size_t i = 0; i < (size_t)n * d; ++i) std::fprintf(out, " %ld", B[i]);
        for (size_t i = 0; i < (size_t)d * n; ++i) std::fprintf(out, " %.17g", P[i]);
      }
      std::fprintf(out, "\n");
    } else if (std::string(kind) == "lift") {
      int m, n, mi;
      if (std::fscanf(in, "%d %d %d", &m, &n, &mi) != 3) return 2;
      std::vector<int64_t> A = read_vec(in, (size_t)m * n), b = read_vec(in, m), l = read_vec(in, n),
                           u = read_vec(in, n), G = read_vec(in, (size_t)mi * n), h = read_vec(in, mi);
      const int N2 = n + mi, M2 = m + mi;
      std::vector<int64_t> A2((size_t)M2 * N2), b2(M2), l2(N2), u2(N2);
      graver_status st = graver_lift_inequalities(m, n, m ? A.data() : nullptr, m ? b.data() : nullptr, l.data(),
                                                  u.data(), mi, G.data(), h.data(), 0, nullptr, A2.data(), b2.data(),
                                                  l2.data(), u2.data(), nullptr);
      std::fprintf(out, "lift %d", (int)st);
      if (st == GRAVER_OK) {
        for (int64_t x : A2) std::fprintf(out, " %ld", x);
        for (int64_t x : b2) std::fprintf(out, " %ld", x);
        for (int64_t x : l2) std::fprintf(out, " %ld", x);
        for (int64_t x : u2) std::fprintf(out, " %ld", x);
      }
      std::fprintf(out, "\n");
    } else {
      return 2;
    }
  }
  std::fclose(in);
  std::fclose(out);
  return 0;
}
