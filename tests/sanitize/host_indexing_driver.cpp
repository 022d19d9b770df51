// Sanitizer driver for the host indexing (test infrastructure).
//
// Reads problems from a case file and builds the indexing of each one
// `repeats` times through the library's C ABI (cb_host_indexing), which runs
// the multithreaded host indexing.  For every problem it prints one line:
// n_dof n_coarse n_objects n_iface, or the error code.  Built with
// AddressSanitizer + UndefinedBehaviorSanitizer or ThreadSanitizer by
// tests/test_host_sanitizers.py.
//
// Case file (native endianness): int32 count, then per problem int32
// n_cells, sub_cells, n_balls, coarse_variant, objects; float64
// centres[3 n_balls], radii[n_balls]; int32 cell_count[n_cells^3].
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "cutbddc.h"

int main(int argc, char** argv) {
  if (argc < 3) {
    std::fprintf(stderr, "usage: %s cases.bin repeats\n", argv[0]);
    return 2;
  }
  const long repeats = std::atol(argv[2]);
  FILE* fh = std::fopen(argv[1], "rb");
  if (!fh) return 2;
  int32_t count = 0;
  if (std::fread(&count, 4, 1, fh) != 1) return 2;
  for (int k = 0; k < count; ++k) {
    int32_t hd[5];
    if (std::fread(hd, 4, 5, fh) != 5) return 2;
    const int N = hd[0], nb = hd[2];
    std::vector<double> centres(3 * (size_t)nb), radii((size_t)nb);
    std::vector<int32_t> cells((size_t)N * N * N);
    if (nb > 0 && (std::fread(centres.data(), 8, centres.size(), fh) != centres.size() ||
                   std::fread(radii.data(), 8, radii.size(), fh) != radii.size()))
      return 2;
    if (std::fread(cells.data(), 4, cells.size(), fh) != cells.size()) return 2;
    cb_problem p{};
    p.n_cells = N;
    p.sub_cells = hd[1];
    p.n_balls = nb;
    p.ball_centres = centres.data();
    p.ball_radii = radii.data();
    p.coarse_variant = hd[3];
    p.objects = hd[4];
    p.weighting = CB_W_STIFFNESS;
    cb_info info{};
    int rc = CB_OK;
    for (long r = 0; r < repeats && rc == CB_OK; ++r) {
      rc = cb_host_indexing(&p, cells.data(), &info, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
      if (rc == CB_OK) {
        std::vector<int64_t> dof((size_t)info.n_dof), optr((size_t)info.n_objects + 1), odofs((size_t)info.n_iface);
        std::vector<int32_t> card((size_t)info.n_dof), coarse((size_t)info.n_objects);
        std::vector<int8_t> otype((size_t)info.n_objects);
        rc = cb_host_indexing(&p, cells.data(), &info, dof.data(), card.data(), optr.data(), odofs.data(),
                              otype.data(), coarse.data());
      }
    }
    if (rc == CB_OK)
      std::printf("%lld %d %d %d\n", (long long)info.n_dof, info.n_coarse, info.n_objects, info.n_iface);
    else
      std::printf("error %d\n", rc);
  }
  // argument errors reported without touching the device
  cb_problem bad{};
  bad.n_cells = 10;
  bad.sub_cells = 4;
  cb_ctx* ctx = nullptr;
  std::printf("setup_error %d\n", cb_setup(&bad, nullptr, &ctx));
  std::fclose(fh);
  return 0;
}
