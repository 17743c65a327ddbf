// The tuner's choices as the library reads them (host side only).  The Python tuner measures
// every plan option set for a shape (Section VI-C's kernel sizes, Section VII's OT depth and
// base) and writes its choices to a JSON cache and, for C callers, to this flat text file,
// one line per tuned shape and no comments:
//
//   <device> <source_hash> <N> <L> <P> <qbits> <log2_n1> <twiddle_mode> <ot_stages> <ot_log2_base> <kernel_path>
//       [<r1> <wg_size> <col_width>]
//
// device is "<arch>:<CUs>CU" (e.g. gfx950:256CU), source_hash the hash of the kernel sources
// the choice was measured with, P the polynomials per call and qbits the width of the largest
// prime; the three tile fields (values per lane and workgroup lanes of the row pass, column
// tile width; 0 = default) are optional.  A line that does not parse is skipped.
#pragma once
#include <cmath>
#include <cstdint>
#include <sstream>
#include <string>
#include <vector>

namespace nttt {

struct TuneEntry {
  std::string device, hash;
  uint32_t N = 0, L = 0, P = 0, qbits = 0;
  int32_t log2_n1 = 0, twiddle_mode = 0, ot_stages = 0, ot_log2_base = 0, kernel_path = 0;
  int32_t r1 = 0, wg_size = 0, col_width = 0;
};

inline std::vector<TuneEntry> parse_tune_file(const std::string& text) {
  std::vector<TuneEntry> out;
  std::istringstream lines(text);
  std::string line;
  while (std::getline(lines, line)) {
    std::istringstream f(line);
    TuneEntry e;
    if (!(f >> e.device >> e.hash >> e.N >> e.L >> e.P >> e.qbits >> e.log2_n1 >> e.twiddle_mode >> e.ot_stages >>
          e.ot_log2_base >> e.kernel_path))
      continue;
    std::vector<std::string> rest;
    std::string tok;
    while (f >> tok) rest.push_back(tok);
    if (rest.size() == 3) {
      std::istringstream t(rest[0] + " " + rest[1] + " " + rest[2]);
      std::string extra;
      if (!(t >> e.r1 >> e.wg_size >> e.col_width) || (t >> extra)) continue;
    } else if (!rest.empty()) {
      continue;
    }
    out.push_back(e);
  }
  return out;
}

// The entry for a plan of N points over L primes of width qbits, used P polynomials per call,
// on `device` with kernels of `hash`: the exact (L, P) entry when there is one, else the
// entry of the same device, kernels, N and width whose work per call L*P is nearest in ratio
// (the choice follows how many vectors one launch covers).  nullptr when none matches.
inline const TuneEntry* pick_tune_entry(const std::vector<TuneEntry>& es, const std::string& device,
                                        const std::string& hash, uint32_t N, uint32_t L, uint32_t P, uint32_t qbits) {
  const TuneEntry* best = nullptr;
  double best_d = 0;
  for (const TuneEntry& e : es) {
    if (e.device != device || e.hash != hash || e.N != N || e.qbits != qbits || e.L == 0 || e.P == 0) continue;
    if (e.L == L && e.P == P) return &e;
    const double d = std::fabs(std::log((double)e.L * e.P) - std::log((double)L * P));
    if (!best || d < best_d) {
      best = &e;
      best_d = d;
    }
  }
  return best;
}

}  // namespace nttt
