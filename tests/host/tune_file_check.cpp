// Host check of the tuning file reader (compiled with g++ by the test suite): lines parse into
// entries, malformed lines are skipped, an exact shape wins, otherwise the nearest work per
// call among entries of the same device, kernels, N and prime width; nothing else matches.
#include <cstdio>
#include <string>

#include "tune_file.hpp"

static long failures = 0;
static void check(bool ok, const char* what) {
  if (!ok && failures++ < 20) std::printf("FAIL %s\n", what);
}

int main() {
  const std::string text =
      "gfx950:256CU abc 65536 45 2 60 6 2 1 10 1\n"
      "gfx950:256CU abc 65536 60 46 60 6 1 0 10 1\n"
      "gfx950:256CU abc 65536 4 1 60 8 1 0 10 1\n"
      "gfx950:256CU old 65536 45 2 60 7 1 0 10 1\n"        // other kernel build
      "gfx950:80CU abc 65536 45 2 60 5 1 0 10 1\n"         // other device
      "gfx950:256CU abc 65536 45 2 62 9 1 0 10 1\n"        // other prime width
      "gfx950:256CU abc 131072 60 2 60 6 1 0 10 1\n"
      "gfx950:256CU abc 65536 45 2 60 6 2 1\n"             // truncated: skipped
      "gfx950:256CU abc 65536 45 2 60 6 2 1 10 1 extra\n"  // one trailing field: skipped
      "gfx950:256CU abc 16384 8 4 60 5 1 0 10 1 4 256 32\n"   // with the tile fields
      "gfx950:256CU abc 16384 8 4 61 5 1 0 10 1 4 256\n"      // two tile fields: skipped
      "gfx950:256CU abc 16384 8 4 62 5 1 0 10 1 4 x 32\n"     // non-numeric tile field: skipped
      "garbage\n";
  const auto es = nttt::parse_tune_file(text);
  check(es.size() == 8, "eight well-formed lines");
  const nttt::TuneEntry* t = nttt::pick_tune_entry(es, "gfx950:256CU", "abc", 16384, 8, 4, 60);
  check(t && t->r1 == 4 && t->wg_size == 256 && t->col_width == 32 && t->log2_n1 == 5, "tile fields");
  t = nttt::pick_tune_entry(es, "gfx950:256CU", "abc", 65536, 45, 2, 60);
  check(t && t->r1 == 0 && t->wg_size == 0 && t->col_width == 0, "tile fields default to zero");
  const nttt::TuneEntry* e = nttt::pick_tune_entry(es, "gfx950:256CU", "abc", 65536, 45, 2, 60);
  check(e && e->log2_n1 == 6 && e->twiddle_mode == 2 && e->ot_stages == 1 && e->ot_log2_base == 10 &&
            e->kernel_path == 1,
        "exact shape");
  e = nttt::pick_tune_entry(es, "gfx950:256CU", "abc", 65536, 60, 40, 60);
  check(e && e->L == 60 && e->P == 46, "nearest work per call (large)");
  e = nttt::pick_tune_entry(es, "gfx950:256CU", "abc", 65536, 3, 1, 60);
  check(e && e->L == 4 && e->P == 1, "nearest work per call (small)");
  e = nttt::pick_tune_entry(es, "gfx950:256CU", "abc", 65536, 45, 2, 62);
  check(e && e->log2_n1 == 9, "prime width is part of the key");
  check(!nttt::pick_tune_entry(es, "gfx950:256CU", "zzz", 65536, 45, 2, 60), "other kernels: no entry");
  check(!nttt::pick_tune_entry(es, "gfx942:304CU", "abc", 65536, 45, 2, 60), "other device: no entry");
  check(!nttt::pick_tune_entry(es, "gfx950:256CU", "abc", 32768, 45, 2, 60), "other N: no entry");
  check(nttt::parse_tune_file("").empty(), "empty file");
  std::printf("%ld failures\n", failures);
  return failures != 0;
}
