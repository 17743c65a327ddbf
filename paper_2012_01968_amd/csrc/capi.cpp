// C ABI of the NTT library: plan construction and the batched entry points.
// Every entry point catches everything; no exception crosses the interface.
#include "ntt_mi355x.h"

#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "crt_math.hpp"
#include "kernels.hpp"
#include "passes.hpp"
#include "plan_life.hpp"
#include "plan_math.hpp"
#include "tune_file.hpp"

#ifndef NTT_SOURCE_HASH
#define NTT_SOURCE_HASH "unknown"
#endif

using nttk::PassArgs;
using nttk::Tw;

namespace {

thread_local std::string g_last_error;

ntt_status fail(ntt_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

ntt_status hip_fail(hipError_t e, const char* where) {
  return fail(NTT_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Makes the plan's device current for the duration of a call and restores the
// caller's device afterwards.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) {
      ok = false;
      return;
    }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

template <typename T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return hipSuccess;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), src.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace

struct ntt_plan_s {
  uint32_t N = 0, logN = 0, L = 0, logN1 = 0;
  int32_t twiddle_mode = NTT_TWIDDLE_TABLE;
  int32_t ot_stages = 0;
  uint32_t ot_log2_base = 10;
  int32_t kernel_path = NTT_PATH_SPLIT;   // SPLIT or FUSED after creation
  int32_t order = NTT_ORDER_BITREV;       // NTT-domain slot order seen by the caller
  int32_t log2_radix = 0;                 // RADIX2 / REGISTER paths: stages per launch
  int32_t word_bits = 64;                 // residue word: 64 (uint64_t) or 32 (uint32_t, q < 2^30)
  uint32_t row_lr = 0, row_nth = 0, col_w = 0;   // split-pass tile shape (0 = built-in default)
  uint32_t debug = 0;                     // split-pass debug modes (NTT_DEBUG at creation)
  uint32_t fused_lag = 4;                 // vectors an XCD queue runs pass 1 ahead of pass 2
  uint32_t fused_grid = 1024;             // persistent workgroups (4 per CU)
  uint32_t* d_ctr = nullptr;              // fused-launch counters: 16 + kMaxFusedVectors words
  std::mutex fused_mu;                    // orders fused launches of this plan across streams
  hipEvent_t fused_ev = nullptr;
  hipStream_t fused_last = nullptr;
  bool fused_pending = false;
  int device = 0;
  bool tuned = false; // options taken from the tuner's file (use_autotune)
  bool fast = false;  // all primes below 2^60 (wider lazy ranges, estimated quotients)
  std::vector<uint64_t> primes, psis;

  uint64_t* d_q = nullptr;
  uint64_t* d_mc = nullptr;   // [L][8] per-prime constants of the split passes
  Tw* d_tw_fwd = nullptr;
  Tw* d_tw_inv = nullptr;
  Tw* d_ot_lo_fwd = nullptr;
  Tw* d_ot_hi_fwd = nullptr;
  Tw* d_ot_lo_inv = nullptr;
  Tw* d_ot_hi_inv = nullptr;
  Tw* d_scale = nullptr;
  uint64_t* d_mu = nullptr;
  uint32_t* d_bits = nullptr;
  // 32-bit plans: Tw32 {w, floor(w 2^32 / q)} tables, {1/N, Psi_inv[1]/N}, primes, floor(2^64 / q)
  void* d_tw32_fwd = nullptr;
  void* d_tw32_inv = nullptr;
  void* d_scale32 = nullptr;
  uint32_t* d_q32 = nullptr;
  uint64_t* d_mu64 = nullptr;

  // RNS <-> integer conversion tables (crt_math.hpp), built and uploaded on first use
  struct Crt {
    std::mutex mu;
    bool ready = false;
    uint32_t W = 0;                 // words of Q
    Tw* pow2 = nullptr;             // [L][kCrtMaxInWords]
    Tw* inv = nullptr;              // [L]
    uint64_t* M = nullptr;          // [L][W]
    uint64_t* kQ = nullptr;         // [L + 1][W + 1]
  } crt;

  // References: the creator's and one per batch that names the plan (plan_life.hpp).
  nttl::RefCount rc;

  // Product scratch (NTT(b) of ntt_polymul_negacyclic), one buffer per stream that has run a
  // product: work on one stream is ordered, so products on different streams never wait for
  // each other and products on one stream reuse the buffer in order.  `ev` marks the last
  // product enqueued with the buffer, which must finish before the buffer is replaced.
  struct StreamScratch {
    hipStream_t stream = nullptr;
    std::mutex mu;
    uint64_t* buf = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
  };
  std::mutex stream_scratch_mu;   // guards the list; each entry has its own lock
  std::vector<std::unique_ptr<StreamScratch>> stream_scratch;

  StreamScratch* scratch_for(hipStream_t st) {
    std::lock_guard<std::mutex> lk(stream_scratch_mu);
    for (auto& s : stream_scratch)
      if (s->stream == st) return s.get();
    stream_scratch.emplace_back(new StreamScratch());
    stream_scratch.back()->stream = st;
    return stream_scratch.back().get();
  }

  ~ntt_plan_s() {
    for (auto& s : stream_scratch) {
      if (s->ev) {
        (void)hipEventSynchronize(s->ev);
        (void)hipEventDestroy(s->ev);
      }
      if (s->buf) (void)hipFree(s->buf);
    }
    if (fused_ev) {
      (void)hipEventSynchronize(fused_ev);
      (void)hipEventDestroy(fused_ev);
    }
    void* ptrs[] = {d_q, d_mc, d_tw_fwd, d_tw_inv, d_ot_lo_fwd, d_ot_hi_fwd, d_ot_lo_inv, d_ot_hi_inv,
                    d_scale, d_mu, d_bits, d_ctr, d_tw32_fwd, d_tw32_inv, d_scale32, d_q32, d_mu64,
                    crt.pow2, crt.inv, crt.M, crt.kQ};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
  }

  PassArgs args(uint64_t* data, uint32_t n_polys, bool inverse, uint32_t limbs = 0) const {
    PassArgs a{};
    a.data = data;
    a.vecs = nullptr;
    a.tw = inverse ? d_tw_inv : d_tw_fwd;
    a.ot_lo = inverse ? d_ot_lo_inv : d_ot_lo_fwd;
    a.ot_hi = inverse ? d_ot_hi_inv : d_ot_hi_fwd;
    a.q = d_q;
    a.mc = d_mc;
    a.scale = d_scale;
    const uint32_t Lu = limbs ? limbs : L;
    a.n_vec = (uint64_t)n_polys * Lu;
    a.P = n_polys;
    a.L = Lu;
    a.logN = logN;
    a.logN1 = logN1;
    a.ot_log2_base = ot_log2_base;
    a.fast = fast ? 1u : 0u;
    a.mu = d_mu;
    a.bits = d_bits;
    a.row_lr = row_lr;
    a.row_nth = row_nth;
    a.col_w = col_w;
    a.debug = debug;
    return a;
  }
  int active_ot() const { return twiddle_mode == NTT_TWIDDLE_OT ? ot_stages : 0; }
  // the paths whose data goes back to global memory after every group of stages
  bool stage_path() const { return kernel_path == NTT_PATH_RADIX2 || kernel_path == NTT_PATH_REGISTER; }
  // forward row stages, key product and inverse row stages in one launch (split plans whose
  // NTT domain is the kernels' bit-reversed one)
  bool fuses_key_rows() const { return !stage_path() && order == NTT_ORDER_BITREV; }
  bool fused_for(uint32_t n_polys) const {
    return kernel_path == NTT_PATH_FUSED && (uint64_t)n_polys * L <= kMaxFusedVectors;
  }
  static constexpr uint64_t kMaxFusedVectors = 1u << 16;
};

// Path of the tuner's flat file: $NTT_TUNE_FILE, else tune_cache.txt next to this library.
static std::string tune_file_path() {
  if (const char* e = std::getenv("NTT_TUNE_FILE")) return e;
  Dl_info info{};
  if (!dladdr(reinterpret_cast<void*>(&ntt_plan_create), &info) || !info.dli_fname) return "";
  std::string lib = info.dli_fname;
  const size_t slash = lib.rfind('/');
  return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/tune_cache.txt";
}

// "<arch>:<CUs>CU" of a device, as the tuner names it.
static std::string device_key(int dev) {
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
  std::string arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  return arch + ":" + std::to_string(prop.multiProcessorCount) + "CU";
}

// Fill the option fields left at zero from the tuner's entry for this shape, if there is one.
static bool apply_tuning(ntt_plan_opts& o, int dev, uint32_t N, const uint64_t* primes, uint32_t L) {
  const std::string path = tune_file_path();
  std::ifstream f(path);
  if (path.empty() || !f) return false;
  std::stringstream text;
  text << f.rdbuf();
  const auto entries = nttt::parse_tune_file(text.str());
  uint64_t qmax = 0;
  for (uint32_t l = 0; l < L; ++l) qmax = std::max(qmax, primes[l]);
  uint32_t qbits = 0;
  while (qbits < 64 && (qmax >> qbits)) ++qbits;
  const uint32_t P = o.tune_polys > 0 ? (uint32_t)o.tune_polys : 1u;
  const nttt::TuneEntry* e = nttt::pick_tune_entry(entries, device_key(dev), NTT_SOURCE_HASH, N, L, P, qbits);
  if (!e) return false;
  if (!o.twiddle_mode && !o.ot_stages && !o.ot_log2_base) {
    o.twiddle_mode = e->twiddle_mode;
    o.ot_stages = e->ot_stages;
    o.ot_log2_base = e->ot_log2_base;
  }
  if (!o.log2_n1) o.log2_n1 = e->log2_n1;
  if (!o.kernel_path) o.kernel_path = e->kernel_path;
  // tile shapes exist for 64-bit plans on the split path
  if (!o.r1 && !o.wg_size && !o.col_width && o.kernel_path == NTT_PATH_SPLIT && o.word_bits != 32) {
    o.r1 = e->r1;
    o.wg_size = e->wg_size;
    o.col_width = e->col_width;
  }
  return true;
}

static ntt_status build_plan(ntt_plan_s* p, uint32_t N, const uint64_t* primes, uint32_t L,
                             const ntt_plan_opts* opts) {
  if (N < 2 || N > (1u << 17) || (N & (N - 1))) return fail(NTT_ERR_N, "N must be a power of two in [2, 2^17]");
  p->N = N;
  p->logN = 0;
  while ((1u << p->logN) < N) ++p->logN;
  p->L = L;

  ntt_plan_opts o{};
  if (opts) o = *opts;
  if (o.reserved != 0) return fail(NTT_ERR_ARG, "the reserved option field must be zero");
  const bool stage_path = o.kernel_path == NTT_PATH_RADIX2 || o.kernel_path == NTT_PATH_REGISTER;
  if (o.use_autotune < 0 || o.use_autotune > 1 || o.tune_polys < 0)
    return fail(NTT_ERR_ARG, "use_autotune must be 0 or 1 and tune_polys non-negative");
  if (o.order != NTT_ORDER_BITREV && o.order != NTT_ORDER_NATURAL)
    return fail(NTT_ERR_ARG, "order must be NTT_ORDER_BITREV or NTT_ORDER_NATURAL");
  p->order = o.order;
  if (o.word_bits != 0 && o.word_bits != 32 && o.word_bits != 64)
    return fail(NTT_ERR_ARG, "word_bits must be 0, 32 or 64");
  p->word_bits = o.word_bits == 32 ? 32 : 64;
  const bool w32 = p->word_bits == 32;
  if (o.use_autotune) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(NTT_ERR_HIP, "hipGetDevice failed");
    p->tuned = apply_tuning(o, dev, N, primes, L);
  }
  if (o.kernel_path < 0 || o.kernel_path > NTT_PATH_REGISTER) return fail(NTT_ERR_ARG, "kernel_path out of range");
  if (o.log2_radix < 0 || o.log2_radix > 5) return fail(NTT_ERR_ARG, "log2_radix must be 0..5");
  if (o.log2_radix && o.kernel_path != NTT_PATH_REGISTER)
    return fail(NTT_ERR_ARG, "log2_radix applies to the NTT_PATH_REGISTER path only");
  if (o.twiddle_mode < 0 || o.twiddle_mode > 2) return fail(NTT_ERR_ARG, "twiddle_mode out of range");
  if (o.ot_stages < 0 || o.ot_stages > 2) return fail(NTT_ERR_ARG, "ot_stages must be 0, 1 or 2");
  if (o.ot_log2_base < 0 || o.ot_log2_base > 16) return fail(NTT_ERR_ARG, "ot_log2_base out of range");
  int mode = o.twiddle_mode;
  if (mode == NTT_TWIDDLE_AUTO) mode = o.ot_stages > 0 ? NTT_TWIDDLE_OT : NTT_TWIDDLE_TABLE;
  p->twiddle_mode = mode;
  p->ot_stages = mode == NTT_TWIDDLE_OT ? (o.ot_stages ? o.ot_stages : 2) : 0;
  p->ot_log2_base = o.ot_log2_base ? (uint32_t)o.ot_log2_base : 10u;
  if (mode == NTT_TWIDDLE_OT && p->ot_log2_base >= p->logN)
    return fail(NTT_ERR_UNSUPPORTED, "OT needs a digit base below N");

  if (w32) {
    // 32-bit words: table twiddles, one or two passes, Algorithm 1's order
    if (mode == NTT_TWIDDLE_OT || stage_path || o.kernel_path == NTT_PATH_FUSED || o.order != NTT_ORDER_BITREV)
      return fail(NTT_ERR_UNSUPPORTED, "32-bit plans take table twiddles, the split path and bit-reversed order");
    p->logN1 = o.log2_n1 == 0 ? (p->logN <= 12 ? 0 : p->logN / 2) : (o.log2_n1 < 0 ? 0 : (uint32_t)o.log2_n1);
    if (!nttk::shape32_supported(p->logN, p->logN1))
      return fail(NTT_ERR_UNSUPPORTED, "no 32-bit kernels for this (N, N1) combination");
  } else if (stage_path) {
    // the ablation paths: table twiddles only, no column/row split
    if (mode == NTT_TWIDDLE_OT) return fail(NTT_ERR_UNSUPPORTED, "the radix-2 and register paths take table twiddles");
    if (o.log2_n1) return fail(NTT_ERR_ARG, "log2_n1 does not apply to the radix-2 and register paths");
    p->logN1 = 0;
    p->log2_radix = o.kernel_path == NTT_PATH_RADIX2 ? 1 : (o.log2_radix ? o.log2_radix : 4);
    if (o.kernel_path == NTT_PATH_REGISTER && p->log2_radix < 2)
      return fail(NTT_ERR_ARG, "the register path takes log2_radix 2..5 (1 is NTT_PATH_RADIX2)");
  } else {
    if (o.log2_n1 == 0) {
      p->logN1 = p->logN <= 12 ? 0 : p->logN / 2;
    } else if (o.log2_n1 < 0) {
      p->logN1 = 0;
    } else {
      p->logN1 = (uint32_t)o.log2_n1;
    }
    if (!nttk::shape_supported(p->logN, p->logN1, p->active_ot()))
      return fail(NTT_ERR_UNSUPPORTED, "no kernels for this (N, N1, OT stages) combination");
  }
  // ---- debug modes of the split passes: NTT_DEBUG holds any of "poison" (LDS filled with a
  // poison pattern before use) and "reverse" (workgroups take their tiles in reverse order)
  if (const char* d = std::getenv("NTT_DEBUG")) {
    const std::string v = d;
    if (v.find("poison") != std::string::npos) p->debug |= nttk::kDebugPoisonLds;
    if (v.find("reverse") != std::string::npos) p->debug |= nttk::kDebugReverseTiles;
  }
  // ---- tile shape of the split passes
  if (o.r1 != 0 && o.r1 != 4 && o.r1 != 8) return fail(NTT_ERR_ARG, "r1 must be 0, 4 or 8");
  if (o.wg_size != 0 && o.wg_size != 64 && o.wg_size != 128 && o.wg_size != 256)
    return fail(NTT_ERR_ARG, "wg_size must be 0, 64, 128 or 256");
  if (o.col_width != 0 && o.col_width != 16 && o.col_width != 32 && o.col_width != 64 && o.col_width != 128 &&
      o.col_width != 256)
    return fail(NTT_ERR_ARG, "col_width must be 0, 16, 32, 64, 128 or 256");
  if (o.r1 || o.wg_size || o.col_width) {
    if (w32 || stage_path || o.kernel_path == NTT_PATH_FUSED)
      return fail(NTT_ERR_UNSUPPORTED, "tile options apply to 64-bit plans on the split path");
    p->row_lr = o.r1 == 4 ? 2u : (o.r1 == 8 ? 3u : 0u);
    p->row_nth = (uint32_t)o.wg_size;
    p->col_w = (uint32_t)o.col_width;
    if (!nttk::tiles_supported(p->logN, p->logN1, p->row_lr, p->row_nth, p->col_w))
      return fail(NTT_ERR_UNSUPPORTED, "col_width needs a column pass with at least that many columns");
  }

  // ---- primes
  p->primes.assign(primes, primes + L);
  {
    std::vector<uint64_t> sorted(p->primes);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      return fail(NTT_ERR_PRIME, "primes must be distinct");
  }
  for (uint32_t l = 0; l < L; ++l) {
    const uint64_t q = p->primes[l];
    if (q <= 2 || q >= (1ull << 62)) return fail(NTT_ERR_PRIME, "prime " + std::to_string(q) + " not in (2, 2^62)");
    if (w32 && q >= (1ull << 30))
      return fail(NTT_ERR_PRIME, "prime " + std::to_string(q) + ": 32-bit words need primes below 2^30");
    if ((q - 1) % (2ull * N)) return fail(NTT_ERR_PRIME, "prime " + std::to_string(q) + " is not 1 mod 2N");
    if (!nttp::is_prime(q)) return fail(NTT_ERR_PRIME, std::to_string(q) + " is not prime");
  }

  p->fast = *std::max_element(p->primes.begin(), p->primes.end()) < (1ull << 60);
  {
    const bool can_fuse = p->fast && p->logN1 != 0 && nttk::fused_supported(p->logN, p->logN1, p->active_ot());
    if (o.kernel_path == NTT_PATH_FUSED && !can_fuse)
      return fail(NTT_ERR_UNSUPPORTED, "the fused path needs primes below 2^60 and a built N1 x N2 shape");
    // AUTO takes the split path: on gfx950 the pass-1 output of a split launch already round-trips
    // through the Infinity Cache, and the fused queue measured slower (see the design notes).
    p->kernel_path = (stage_path || w32) ? (w32 ? NTT_PATH_SPLIT : o.kernel_path)
                                : (o.kernel_path == NTT_PATH_FUSED && can_fuse) ? NTT_PATH_FUSED : NTT_PATH_SPLIT;
    if (const char* e = std::getenv("NTT_FUSED_LAG")) p->fused_lag = (uint32_t)std::max(1, std::atoi(e));
    if (const char* e = std::getenv("NTT_FUSED_GRID")) p->fused_grid = (uint32_t)std::max(1, std::atoi(e));
  }

  // ---- tables (host), one worker per block of limbs
  const size_t NN = N;
  const uint32_t b = p->ot_log2_base;
  const bool want_ot = b < p->logN;
  const size_t B = want_ot ? (size_t)1 << b : 0, H = want_ot ? NN >> b : 0;
  std::vector<Tw> tw_fwd(L * NN), tw_inv(L * NN), ot_lo_f(L * B), ot_hi_f(L * H), ot_lo_i(L * B), ot_hi_i(L * H),
      scale(2 * (size_t)L);
  std::vector<uint64_t> mu(L), psis(L);
  std::vector<uint32_t> bits(L);
  std::vector<int> bad(L, 0);
  // 32-bit tables: {w, floor(w 2^32 / q)} per entry, packed as one uint64 (w in the low half)
  std::vector<uint64_t> tw32_f(w32 ? L * NN : 0), tw32_i(w32 ? L * NN : 0), scale32(w32 ? 2 * (size_t)L : 0),
      mu64(w32 ? L : 0);
  std::vector<uint32_t> q32(w32 ? L : 0);
  auto pack32 = [](uint64_t w, uint64_t q) { return w | ((uint64_t)(((nttp::u128)w << 32) / q) << 32); };

  auto work = [&](uint32_t l0, uint32_t l1) {
    std::vector<uint64_t> pw(NN), pwi(NN);
    for (uint32_t l = l0; l < l1; ++l) {
      const uint64_t q = p->primes[l];
      const uint64_t psi = nttp::smallest_primitive_root(q, N);
      if (!psi) {
        bad[l] = 1;
        continue;
      }
      psis[l] = psi;
      const uint64_t psi_inv = nttp::powmod(psi, q - 2, q);
      pw[0] = pwi[0] = 1;
      for (size_t e = 1; e < NN; ++e) {
        pw[e] = nttp::mulmod(pw[e - 1], psi, q);
        pwi[e] = nttp::mulmod(pwi[e - 1], psi_inv, q);
      }
      Tw* tf = &tw_fwd[l * NN];
      Tw* ti = &tw_inv[l * NN];
      for (size_t i = 0; i < NN; ++i) {
        const uint32_t e = nttp::bitrev((uint32_t)i, (int)p->logN);
        tf[i] = Tw{pw[e], nttp::shoup_companion(pw[e], q)};
        ti[i] = Tw{pwi[e], nttp::shoup_companion(pwi[e], q)};
      }
      for (size_t k = 0; k < B; ++k) {
        ot_lo_f[l * B + k] = Tw{pw[k], nttp::shoup_companion(pw[k], q)};
        ot_lo_i[l * B + k] = Tw{pwi[k], nttp::shoup_companion(pwi[k], q)};
      }
      for (size_t h = 0; h < H; ++h) {
        const uint64_t wf = pw[h << b], wi = pwi[h << b];
        ot_hi_f[l * H + h] = Tw{wf, nttp::shoup_companion(wf, q)};
        ot_hi_i[l * H + h] = Tw{wi, nttp::shoup_companion(wi, q)};
      }
      const uint64_t n_inv = nttp::powmod(N % q, q - 2, q);
      const uint64_t w1n = nttp::mulmod(ti[N > 1 ? 1 : 0].w, n_inv, q);
      scale[2 * l] = Tw{n_inv, nttp::shoup_companion(n_inv, q)};
      scale[2 * l + 1] = Tw{w1n, nttp::shoup_companion(w1n, q)};
      uint32_t s = 0;
      while (s < 64 && (q >> s)) ++s;
      bits[l] = s;
      mu[l] = (uint64_t)(((nttp::u128)1 << (2 * s)) / q);
      if (w32) {
        for (size_t i = 0; i < NN; ++i) {
          tw32_f[l * NN + i] = pack32(tf[i].w, q);
          tw32_i[l * NN + i] = pack32(ti[i].w, q);
        }
        scale32[2 * l] = pack32(n_inv, q);
        scale32[2 * l + 1] = pack32(w1n, q);
        q32[l] = (uint32_t)q;
        mu64[l] = (uint64_t)((((nttp::u128)1) << 64) / q);
      }
    }
  };
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const uint32_t workers = (uint64_t)L * NN >= (1u << 18) ? std::min<uint32_t>(hw, L) : 1u;
  if (workers <= 1) {
    work(0, L);
  } else {
    std::vector<std::thread> th;
    for (uint32_t w = 0; w < workers; ++w)
      th.emplace_back(work, (uint32_t)((uint64_t)L * w / workers), (uint32_t)((uint64_t)L * (w + 1) / workers));
    for (auto& t : th) t.join();
  }
  for (uint32_t l = 0; l < L; ++l)
    if (bad[l]) return fail(NTT_ERR_PRIME, "no primitive 2N-th root found mod " + std::to_string(p->primes[l]));
  p->psis = psis;
  std::vector<uint64_t> mod_consts(8 * (size_t)L, 0);
  for (uint32_t l = 0; l < L; ++l) {
    const uint64_t q = p->primes[l];
    uint64_t* c = &mod_consts[8 * (size_t)l];
    c[0] = q;
    c[1] = q << 1;
    c[2] = q << 2;
    c[3] = 0 - q;
    c[4] = 0 - (q << 1);
    c[5] = 0 - (q << 2);
    c[6] = 0 - (q << 3);
    c[7] = nttk::quot_estimate_consts(q);
  }

  if (w32) {   // a 32-bit plan keeps only its 32-bit tables on the device
    for (auto* v : {&tw_fwd, &tw_inv, &ot_lo_f, &ot_hi_f, &ot_lo_i, &ot_hi_i, &scale}) std::vector<Tw>().swap(*v);
  }
  if (hipGetDevice(&p->device) != hipSuccess) return fail(NTT_ERR_HIP, "hipGetDevice failed");
  hipError_t e;
  {
    uint64_t* f = nullptr;
    uint64_t* i = nullptr;
    uint64_t* sc = nullptr;
    if ((e = upload(&f, tw32_f)) != hipSuccess || (p->d_tw32_fwd = f, (e = upload(&i, tw32_i)) != hipSuccess) ||
        (p->d_tw32_inv = i, (e = upload(&sc, scale32)) != hipSuccess) ||
        (p->d_scale32 = sc, (e = upload(&p->d_q32, q32)) != hipSuccess) || (e = upload(&p->d_mu64, mu64)) != hipSuccess) {
      if (e == hipErrorOutOfMemory) return fail(NTT_ERR_NOMEM, "device allocation of plan tables failed");
      return hip_fail(e, "uploading plan tables");
    }
  }
  if ((e = upload(&p->d_q, p->primes)) != hipSuccess || (e = upload(&p->d_mc, mod_consts)) != hipSuccess ||
      (e = upload(&p->d_tw_fwd, tw_fwd)) != hipSuccess ||
      (e = upload(&p->d_tw_inv, tw_inv)) != hipSuccess || (e = upload(&p->d_ot_lo_fwd, ot_lo_f)) != hipSuccess ||
      (e = upload(&p->d_ot_hi_fwd, ot_hi_f)) != hipSuccess || (e = upload(&p->d_ot_lo_inv, ot_lo_i)) != hipSuccess ||
      (e = upload(&p->d_ot_hi_inv, ot_hi_i)) != hipSuccess || (e = upload(&p->d_scale, scale)) != hipSuccess ||
      (e = upload(&p->d_mu, mu)) != hipSuccess || (e = upload(&p->d_bits, bits)) != hipSuccess) {
    if (e == hipErrorOutOfMemory) return fail(NTT_ERR_NOMEM, "device allocation of plan tables failed");
    return hip_fail(e, "uploading plan tables");
  }
  if (p->kernel_path == NTT_PATH_FUSED) {
    const size_t words = 16 + ntt_plan_s::kMaxFusedVectors;
    if ((e = hipMalloc(reinterpret_cast<void**>(&p->d_ctr), words * sizeof(uint32_t))) != hipSuccess)
      return e == hipErrorOutOfMemory ? fail(NTT_ERR_NOMEM, "counter allocation failed") : hip_fail(e, "hipMalloc");
    if ((e = hipMemset(p->d_ctr, 0, words * sizeof(uint32_t))) != hipSuccess) return hip_fail(e, "hipMemset");
    if ((e = hipEventCreateWithFlags(&p->fused_ev, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "hipEventCreate");
  }
  return NTT_OK;
}

// Free a plan whose last reference is gone: wait for everything queued on its device (which
// includes every launch that reads its tables), then release its memory.
static void plan_finalise(ntt_plan_t plan) {
  DeviceGuard g(plan->device);
  (void)hipDeviceSynchronize();
  delete plan;
}

static void plan_release(ntt_plan_t plan) {
  if (plan->rc.release()) plan_finalise(plan);
}

// Both passes in one persistent launch.  Launches of one plan share its counter block, so a
// launch on a stream other than the previous one waits for that previous launch.
static hipError_t launch_fused(ntt_plan_t plan, uint64_t* data, uint32_t n_polys, bool inverse, hipStream_t st) {
  std::lock_guard<std::mutex> lk(plan->fused_mu);
  hipError_t e;
  if (plan->fused_pending && plan->fused_last != st && (e = hipStreamWaitEvent(st, plan->fused_ev, 0)) != hipSuccess)
    return e;
  e = nttk::launch_fused(plan->args(data, n_polys, inverse), plan->active_ot(), inverse, plan->d_ctr, n_polys,
                         plan->fused_lag, plan->fused_grid, st);
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(plan->fused_ev, st)) != hipSuccess) return e;
  plan->fused_last = st;
  plan->fused_pending = true;
  return hipSuccess;
}

// The transform proper (bit-reversed NTT domain), without the natural-order permutation.
// Every pass of one direction over the vectors of `a` (dense or list), by the plan's path.
static hipError_t enqueue_direction(ntt_plan_t plan, const PassArgs& a, bool inverse, hipStream_t st) {
  if (plan->stage_path()) return nttk::launch_stage_groups(a, plan->log2_radix, inverse, st);
  return inverse ? nttk::launch_inverse(a, plan->active_ot(), st) : nttk::launch_forward(a, plan->active_ot(), st);
}

static hipError_t transform_brv(ntt_plan_t plan, uint64_t* data, uint32_t n_polys, bool inverse, hipStream_t st,
                                uint32_t limbs) {
  if ((limbs == 0 || limbs == plan->L) && plan->fused_for(n_polys)) return launch_fused(plan, data, n_polys, inverse, st);
  return enqueue_direction(plan, plan->args(data, n_polys, inverse, limbs), inverse, st);
}

// A transform as the caller sees it: natural-order plans permute the NTT-domain slots after
// the forward transform and before the inverse.
static hipError_t transform(ntt_plan_t plan, uint64_t* data, uint32_t n_polys, bool inverse, hipStream_t st,
                            uint32_t limbs = 0) {
  hipError_t e;
  const bool nat = plan->order == NTT_ORDER_NATURAL;
  if (nat && inverse && (e = nttk::launch_brv_permute(plan->args(data, n_polys, true, limbs), st)) != hipSuccess)
    return e;
  if ((e = transform_brv(plan, data, n_polys, inverse, st, limbs)) != hipSuccess) return e;
  if (nat && !inverse && (e = nttk::launch_brv_permute(plan->args(data, n_polys, false, limbs), st)) != hipSuccess)
    return e;
  return hipSuccess;
}

static ntt_status check_plan(ntt_plan_t plan) {
  if (!plan) return fail(NTT_ERR_ARG, "plan is NULL");
  if (plan->rc.owner_gone.load(std::memory_order_relaxed))
    return fail(NTT_ERR_ARG, "plan was destroyed (only the batches that name it may still run it)");
  return NTT_OK;
}

static ntt_status check_data_words(ntt_plan_t plan, const void* ptr, uint32_t n_polys, int word_bits);

static ntt_status check_data(ntt_plan_t plan, const void* ptr, uint32_t n_polys) {
  return check_data_words(plan, ptr, n_polys, 64);
}

static ntt_status check_data_words(ntt_plan_t plan, const void* ptr, uint32_t n_polys, int word_bits) {
  if (ntt_status s = check_plan(plan)) return s;
  if (plan->word_bits != word_bits)
    return fail(NTT_ERR_ARG, plan->word_bits == 32 ? "the plan holds 32-bit words: use the _u32 entry points"
                                                   : "the plan holds 64-bit words: use the uint64_t entry points");
  if (!ptr) return fail(NTT_ERR_ARG, "data pointer is NULL");
  if (reinterpret_cast<uintptr_t>(ptr) & 15) return fail(NTT_ERR_ARG, "data pointer must be 16-byte aligned");
  if (n_polys == 0) return fail(NTT_ERR_ARG, "n_polys must be at least 1");
  // every pass launches at most N/16 + 1 workgroups per vector; keep the grid below 2^31
  const uint64_t n_vec = (uint64_t)n_polys * plan->L;
  if (n_vec * ((uint64_t)plan->N / 16 + 1) >= (1ull << 31)) return fail(NTT_ERR_ARG, "batch too large for one launch");
  return NTT_OK;
}

static ntt_status check_product(ntt_plan_t plan, const uint64_t* d_a, const uint64_t* d_b, const uint64_t* d_c,
                                uint32_t n_polys) {
  ntt_status s;
  if ((s = check_data(plan, d_a, n_polys)) != NTT_OK || (s = check_data(plan, d_b, n_polys)) != NTT_OK ||
      (s = check_data(plan, d_c, n_polys)) != NTT_OK)
    return s;
  if (d_c == d_b) return fail(NTT_ERR_ARG, "d_c must not alias d_b");
  return NTT_OK;
}

// The launches of c = a * b with NTT(b) placed in `tmp` (n_polys*L*N words of device memory
// that nothing else uses until they complete).  Split plans: NTT(b) into tmp (first pass out
// of place), a's forward column pass out of place into c, the row passes with the product by
// NTT(b) in one launch, and the inverse column pass; a single-pass size does the whole
// product in that launch.  Fused-path plans: copies, both transforms, the element-wise
// product and the inverse as separate launches.  Allocates nothing.
static hipError_t polymul_enqueue(ntt_plan_t plan, const uint64_t* d_a, const uint64_t* d_b, uint64_t* d_c,
                                  uint32_t n_polys, uint64_t* tmp, hipStream_t st) {
  hipError_t e;
  const int ot = plan->active_ot();
  if (plan->kernel_path == NTT_PATH_SPLIT) {
    PassArgs fb = plan->args(tmp, n_polys, false);
    PassArgs fa = plan->args(d_c, n_polys, false);
    const PassArgs ia = plan->args(d_c, n_polys, true);
    fb.src = d_b;
    fa.src = d_a;
    fa.key = tmp;
    if (plan->logN1) {
      PassArgs fa_col = fa;
      fa_col.key = nullptr;
      fa.src = nullptr;   // the row launch reads c, which the column pass wrote
      PassArgs fb_row = fb;
      fb_row.src = nullptr;
      if ((e = nttk::launch_forward_pass(fb, ot, 0, st)) != hipSuccess ||
          (e = nttk::launch_forward_pass(fb_row, ot, 1, st)) != hipSuccess ||
          (e = nttk::launch_forward_pass(fa_col, ot, 0, st)) != hipSuccess ||
          (e = nttk::launch_mul_rows(fa, ia, ot, st)) != hipSuccess ||
          (e = nttk::launch_inverse_pass(ia, ot, 1, st)) != hipSuccess)
        return e;
      return hipSuccess;
    }
    if ((e = nttk::launch_forward_pass(fb, ot, 0, st)) != hipSuccess ||
        (e = nttk::launch_mul_rows(fa, ia, ot, st)) != hipSuccess)
      return e;
    return hipSuccess;
  }
  const size_t bytes = (size_t)n_polys * plan->L * plan->N * sizeof(uint64_t);
  if (d_c != d_a && (e = hipMemcpyAsync(d_c, d_a, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(tmp, d_b, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
  if ((e = transform_brv(plan, d_c, n_polys, false, st, 0)) != hipSuccess ||
      (e = transform_brv(plan, tmp, n_polys, false, st, 0)) != hipSuccess ||
      (e = nttk::launch_pointwise(d_c, tmp, d_c, plan->d_q, plan->d_mu, plan->d_bits,
                                  (uint64_t)n_polys * plan->L * plan->N, plan->logN, plan->L, st)) != hipSuccess ||
      (e = transform_brv(plan, d_c, n_polys, true, st, 0)) != hipSuccess)
    return e;
  return hipSuccess;
}

// ---------------------------------------------------------------- batches

struct ntt_batch_s {
  struct Group {                        // every vector of the jobs that share one plan
    ntt_plan_t plan = nullptr;
    uint64_t off_fwd = 0, off_key = 0, off_inv = 0, off_full = 0;   // positions in the descriptor arena
    uint64_t n_fwd = 0, n_key = 0, n_inv = 0, n_full = 0;
  };
  std::vector<ntt_job> jobs;
  std::vector<Group> groups;
  std::vector<ntt_plan_t> held;         // one reference on every distinct plan of the jobs
  int device = 0;
  nttk::VecDesc* d_desc = nullptr;      // descriptor arena (device)
  nttk::VecDesc* h_desc = nullptr;      // pinned staging copy of the arena
  uint64_t cap = 0;                     // capacity of both, in descriptors
  hipEvent_t used = nullptr;            // last run that read the arena
  hipEvent_t uploaded = nullptr;        // last copy out of the staging buffer
  bool used_pending = false, upload_pending = false;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // NTT_BATCH_GRAPH_BRANCHED: its own graph, the streams the branches are captured on and the
  // fork / join events (created on first use, kept for the batch's life)
  hipGraph_t graph_br = nullptr;
  hipGraphExec_t exec_br = nullptr;
  std::vector<hipStream_t> branch_streams;
  std::vector<hipEvent_t> branch_events;   // [0]: fork; [1 + k]: join of branch k + 1
  static constexpr int kBranches = 4;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (exec_br) (void)hipGraphExecDestroy(exec_br);
    if (graph_br) (void)hipGraphDestroy(graph_br);
    exec = nullptr;
    graph = nullptr;
    exec_br = nullptr;
    graph_br = nullptr;
  }

  ~ntt_batch_s() {
    for (hipEvent_t ev : {used, uploaded}) {
      if (!ev) continue;
      (void)hipEventSynchronize(ev);
      (void)hipEventDestroy(ev);
    }
    drop_graph();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    for (hipStream_t bs : branch_streams) (void)hipStreamDestroy(bs);
    for (hipEvent_t ev : branch_events) (void)hipEventDestroy(ev);
    if (d_desc) (void)hipFree(d_desc);
    if (h_desc) (void)hipHostFree(h_desc);
    hold({});
  }

  // Hold references on exactly `plans` (the distinct plans of the current jobs); a plan whose
  // last reference this drops is finalised.
  void hold(const std::vector<ntt_plan_t>& plans) {
    const auto last = nttl::rehold(held, plans, [](ntt_plan_t p) -> nttl::RefCount& { return p->rc; });
    held = plans;
    for (ntt_plan_t p : last) plan_finalise(p);
  }

  const nttk::VecDesc* at(uint64_t off) const { return d_desc + off; }

  // Enqueue the grouped work: all forward vector lists, then the key products, then all
  // inverse lists.
  PassArgs list_args(const Group& g, uint64_t off, uint64_t n, bool inverse) const {
    PassArgs a = g.plan->args(nullptr, 1, inverse);
    a.vecs = at(off);
    a.n_vec = n;
    a.P = 1;
    a.L = g.plan->L;
    return a;
  }

  // Enqueue the grouped work in three phases over all plans: forward transforms, then key
  // products, then inverse transforms.  Vectors of jobs that do all three ("full") take the
  // forward column pass in phase 0, the row passes with the key product (one launch) in
  // phase 1 and the inverse column pass in phase 2; a single-pass size does it all in phase 1.
  hipError_t grouped(hipStream_t st) const {
    for (int phase = 0; phase < 3; ++phase) {
      for (const Group& g : groups) {
        const hipError_t e = group_phase(g, phase, st);
        if (e != hipSuccess) return e;
      }
    }
    return hipSuccess;
  }

  // Phase `phase` (0 forward, 1 key products, 2 inverse) of one plan's vectors.
  hipError_t group_phase(const Group& g, int phase, hipStream_t st) const {
    const int ot = g.plan->active_ot();
    const bool split = g.plan->logN1 != 0;
    hipError_t e = hipSuccess;
    if (phase == 1) {
      if (g.n_key &&
          (e = nttk::launch_pointwise_list(at(g.off_key), g.n_key, g.plan->logN, g.plan->d_q, g.plan->d_mu,
                                           g.plan->d_bits, st)) != hipSuccess)
        return e;
      if (g.n_full &&
          (e = nttk::launch_mul_rows(list_args(g, g.off_full, g.n_full, false),
                                     list_args(g, g.off_full, g.n_full, true), ot, st)) != hipSuccess)
        return e;
      return hipSuccess;
    }
    const bool inv = phase == 2;
    const uint64_t n = inv ? g.n_inv : g.n_fwd;
    if (n) {
      const PassArgs a = list_args(g, inv ? g.off_inv : g.off_fwd, n, inv);
      const bool nat = g.plan->order == NTT_ORDER_NATURAL;
      if (nat && inv && (e = nttk::launch_brv_permute(a, st)) != hipSuccess) return e;
      if ((e = enqueue_direction(g.plan, a, inv, st)) != hipSuccess) return e;
      if (nat && !inv && (e = nttk::launch_brv_permute(a, st)) != hipSuccess) return e;
    }
    if (g.n_full && split) {
      const PassArgs a = list_args(g, g.off_full, g.n_full, inv);
      if ((e = inv ? nttk::launch_inverse_pass(a, ot, 1, st) : nttk::launch_forward_pass(a, ot, 0, st)) !=
          hipSuccess)
        return e;
    }
    return hipSuccess;
  }

  // Work of a group, in butterflies: what the branches are balanced by.
  static double group_work(const Group& g) {
    const double vecs = (double)(g.n_fwd + g.n_inv + 2 * g.n_full) + 0.1 * (double)g.n_key;
    return vecs * (double)g.plan->N * (double)g.plan->logN;
  }

  // Branch of each group: groups sorted by work, each to the least loaded of the branches.
  std::vector<int> branch_of_groups(int nb) const {
    std::vector<size_t> order(groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::sort(order.begin(), order.end(),
              [&](size_t x, size_t y) { return group_work(groups[x]) > group_work(groups[y]); });
    std::vector<double> load(nb, 0.0);
    std::vector<int> br(groups.size(), 0);
    for (size_t i : order) {
      const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      br[i] = k;
      load[k] += group_work(groups[i]);
    }
    return br;
  }

  // The groups' chains as independent branches: branch 0 on `st`, branches 1.. on the
  // batch's own streams after a fork event, joined back into `st` by one event each.  Every
  // group's vectors are its own (jobs may not overlap), so the branches need no ordering
  // among themselves; on the device, small sizes then run beside the large ones.
  hipError_t branched(hipStream_t st) {
    const int nb = (int)std::min<size_t>(kBranches, groups.size());
    hipError_t e;
    while ((int)branch_streams.size() < nb - 1) {
      hipStream_t s = nullptr;
      if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return e;
      branch_streams.push_back(s);
    }
    while ((int)branch_events.size() < nb) {
      hipEvent_t ev = nullptr;
      if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
      branch_events.push_back(ev);
    }
    const std::vector<int> br = branch_of_groups(nb);
    if (nb > 1) {
      if ((e = hipEventRecord(branch_events[0], st)) != hipSuccess) return e;
      for (int k = 1; k < nb; ++k)
        if ((e = hipStreamWaitEvent(branch_streams[k - 1], branch_events[0], 0)) != hipSuccess) return e;
    }
    for (int k = 0; k < nb; ++k) {
      hipStream_t s = k ? branch_streams[k - 1] : st;
      for (size_t i = 0; i < groups.size(); ++i) {
        if (br[i] != k) continue;
        for (int phase = 0; phase < 3; ++phase)
          if ((e = group_phase(groups[i], phase, s)) != hipSuccess) return e;
      }
    }
    for (int k = 1; k < nb; ++k) {
      if ((e = hipEventRecord(branch_events[k], branch_streams[k - 1])) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(st, branch_events[k], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
  }
};

// Validate the jobs and fill the batch's groups and descriptors (host side).
static ntt_status plan_batch(ntt_batch_s* b, const ntt_job* jobs, uint32_t n_jobs, std::vector<nttk::VecDesc>& desc) {
  if (!jobs || n_jobs == 0) return fail(NTT_ERR_ARG, "jobs must be a non-empty array");
  std::vector<ntt_job> js(jobs, jobs + n_jobs);
  std::vector<ntt_plan_t> plans;
  for (uint32_t j = 0; j < n_jobs; ++j) {
    const ntt_job& job = js[j];
    if (!job.plan || !job.d_data) return fail(NTT_ERR_ARG, "job " + std::to_string(j) + ": NULL plan or data");
    if (job.plan->rc.owner_gone.load(std::memory_order_relaxed))
      return fail(NTT_ERR_ARG, "job " + std::to_string(j) + ": plan was destroyed");
    if (job.plan->word_bits != 64)
      return fail(NTT_ERR_UNSUPPORTED, "job " + std::to_string(j) + ": batches take 64-bit plans");
    if (reinterpret_cast<uintptr_t>(job.d_data) & 15) return fail(NTT_ERR_ARG, "job data must be 16-byte aligned");
    if (job.n_polys == 0 || job.n_limbs > job.plan->L || job.reserved)
      return fail(NTT_ERR_ARG, "job " + std::to_string(j) + ": bad n_polys, n_limbs or reserved field");
    if (job.op == 0 || job.op > (NTT_OP_FORWARD | NTT_OP_INVERSE | NTT_OP_MULKEY))
      return fail(NTT_ERR_ARG, "job " + std::to_string(j) + ": bad op");
    if ((job.op & NTT_OP_MULKEY) && (!job.d_key || (reinterpret_cast<uintptr_t>(job.d_key) & 15)))
      return fail(NTT_ERR_ARG, "job " + std::to_string(j) + ": MULKEY needs a 16-byte aligned key");
    if (job.plan->device != b->device) return fail(NTT_ERR_ARG, "jobs span several devices");
    if (std::find(plans.begin(), plans.end(), job.plan) == plans.end()) plans.push_back(job.plan);
  }
  std::vector<ntt_batch_s::Group> groups;
  desc.clear();
  for (ntt_plan_t plan : plans) {
    ntt_batch_s::Group g;
    g.plan = plan;
    std::vector<nttk::VecDesc> fwd, key, inv, full;
    // limb-major: the polynomials of one limb are adjacent, so launches meet its twiddles together
    for (uint32_t l = 0; l < plan->L; ++l) {
      for (const ntt_job& job : js) {
        if (job.plan != plan) continue;
        const uint32_t lim = job.n_limbs ? job.n_limbs : plan->L;
        if (l >= lim) continue;
        for (uint32_t p = 0; p < job.n_polys; ++p) {
          nttk::VecDesc d{job.d_data + ((uint64_t)p * lim + l) * plan->N, nullptr, l, 0};
          if (job.op & NTT_OP_MULKEY) d.key = job.d_key + (uint64_t)l * plan->N;
          // forward, key product and inverse in the fused row launch; natural-order plans take
          // their keys in natural order, so they run the three steps as separate lists instead
          if (job.op == (NTT_OP_FORWARD | NTT_OP_MULKEY | NTT_OP_INVERSE) && plan->fuses_key_rows()) {
            full.push_back(d);
            continue;
          }
          if (job.op & NTT_OP_FORWARD) fwd.push_back(d);
          if (job.op & NTT_OP_INVERSE) inv.push_back(d);
          if (job.op & NTT_OP_MULKEY) key.push_back(d);
        }
      }
    }
    for (auto* list : {&fwd, &key, &inv, &full})
      if (list->size() * ((uint64_t)plan->N / 16 + 1) >= (1ull << 31)) return fail(NTT_ERR_ARG, "batch too large for one launch");
    g.off_fwd = desc.size();
    g.n_fwd = fwd.size();
    desc.insert(desc.end(), fwd.begin(), fwd.end());
    g.off_key = desc.size();
    g.n_key = key.size();
    desc.insert(desc.end(), key.begin(), key.end());
    g.off_inv = desc.size();
    g.n_inv = inv.size();
    desc.insert(desc.end(), inv.begin(), inv.end());
    g.off_full = desc.size();
    g.n_full = full.size();
    desc.insert(desc.end(), full.begin(), full.end());
    groups.push_back(g);
  }
  b->jobs.swap(js);
  b->groups.swap(groups);
  b->hold(plans);
  return NTT_OK;
}

// Copy descriptors into the arena on `st`, behind the batch's last run; the arena grows
// (after that run has finished) when the new set does not fit.
static ntt_status upload_batch(ntt_batch_s* b, const std::vector<nttk::VecDesc>& desc, hipStream_t st) {
  hipError_t e;
  if (desc.size() > b->cap) {
    if (b->used_pending && (e = hipEventSynchronize(b->used)) != hipSuccess) return hip_fail(e, "waiting for batch");
    if (b->upload_pending && (e = hipEventSynchronize(b->uploaded)) != hipSuccess)
      return hip_fail(e, "waiting for batch upload");
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    b->d_desc = b->h_desc = nullptr;
    b->cap = 0;
    const uint64_t cap = std::max<uint64_t>(desc.size(), 256);
    if ((e = hipMalloc(reinterpret_cast<void**>(&b->d_desc), cap * sizeof(nttk::VecDesc))) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void**>(&b->h_desc), cap * sizeof(nttk::VecDesc), 0)) != hipSuccess)
      return e == hipErrorOutOfMemory ? fail(NTT_ERR_NOMEM, "descriptor allocation failed")
                                      : hip_fail(e, "descriptor allocation");
    b->cap = cap;
  }
  b->drop_graph();
  if (desc.empty()) return NTT_OK;
  // the staging buffer may still feed the previous copy; the arena may still feed the last run
  if (b->upload_pending && (e = hipEventSynchronize(b->uploaded)) != hipSuccess)
    return hip_fail(e, "waiting for batch upload");
  if (b->used_pending && (e = hipStreamWaitEvent(st, b->used, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  std::copy(desc.begin(), desc.end(), b->h_desc);
  if ((e = hipMemcpyAsync(b->d_desc, b->h_desc, desc.size() * sizeof(nttk::VecDesc), hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipEventRecord(b->uploaded, st)) != hipSuccess)
    return hip_fail(e, "uploading batch descriptors");
  b->upload_pending = true;
  return NTT_OK;
}

namespace nttk {
// One-pass device copy of n16 16-byte vectors (calib.hip).
hipError_t launch_copy16(const void* src, void* dst, uint64_t n16, hipStream_t st);
}  // namespace nttk

extern "C" {

ntt_status ntt_plan_create(ntt_plan_t* out, uint32_t N, const uint64_t* primes, uint32_t L,
                           const ntt_plan_opts* opts) {
  try {
    if (!out) return fail(NTT_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!primes || L == 0) return fail(NTT_ERR_ARG, "primes must be a non-empty array");
    ntt_plan_s* p = new (std::nothrow) ntt_plan_s();
    if (!p) return fail(NTT_ERR_NOMEM, "host allocation failed");
    const ntt_status s = build_plan(p, N, primes, L, opts);
    if (s != NTT_OK) {
      delete p;
      return s;
    }
    *out = p;
    return NTT_OK;
  } catch (const std::bad_alloc&) {
    return fail(NTT_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_plan_create");
  }
}

ntt_status ntt_plan_destroy(ntt_plan_t plan) {
  try {
    if (!plan) return NTT_OK;
    switch (plan->rc.release_owner()) {
      case nttl::RefCount::kAlreadyGone:
        return fail(NTT_ERR_ARG, "plan destroyed twice");
      case nttl::RefCount::kLast:
        plan_finalise(plan);
        break;
      case nttl::RefCount::kStillHeld:   // a batch still names it: freed when the last one lets go
        break;
    }
    return NTT_OK;
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_plan_destroy");
  }
}

ntt_status ntt_plan_get_roots(ntt_plan_t plan, uint64_t* psi_out) {
  if (ntt_status s = check_plan(plan)) return s;
  if (!psi_out) return fail(NTT_ERR_ARG, "NULL argument");
  std::memcpy(psi_out, plan->psis.data(), plan->L * sizeof(uint64_t));
  return NTT_OK;
}

int32_t ntt_plan_log2_radix(ntt_plan_t plan) {
  if (check_plan(plan) != NTT_OK) return -1;
  return plan->log2_radix;
}

int32_t ntt_plan_order(ntt_plan_t plan) {
  if (check_plan(plan) != NTT_OK) return -1;
  return plan->order;
}

ntt_status ntt_plan_get_info(ntt_plan_t plan, uint32_t* N, uint32_t* L, uint32_t* log2_n1, int32_t* twiddle_mode,
                             int32_t* ot_stages, int32_t* kernel_path) {
  if (ntt_status s = check_plan(plan)) return s;
  if (N) *N = plan->N;
  if (L) *L = plan->L;
  if (log2_n1) *log2_n1 = plan->logN1;
  if (twiddle_mode) *twiddle_mode = plan->twiddle_mode;
  if (ot_stages) *ot_stages = plan->ot_stages;
  if (kernel_path) *kernel_path = plan->kernel_path;
  return NTT_OK;
}

ntt_status ntt_plan_get_tiles(ntt_plan_t plan, int32_t* r1, int32_t* wg_size, int32_t* col_width) {
  if (ntt_status s = check_plan(plan)) return s;
  if (r1) *r1 = (int32_t)plan->row_lr ? (1 << plan->row_lr) : 0;
  if (wg_size) *wg_size = (int32_t)plan->row_nth;
  if (col_width) *col_width = (int32_t)plan->col_w;
  return NTT_OK;
}

ntt_status ntt_forward(ntt_plan_t plan, uint64_t* d_data, uint32_t n_polys, void* stream) {
  try {
    ntt_status s = check_data(plan, d_data, n_polys);
    if (s != NTT_OK) return s;
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
    const hipError_t e = transform(plan, d_data, n_polys, false, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? NTT_OK : hip_fail(e, "ntt_forward launch");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_forward");
  }
}

int32_t ntt_plan_tuned(ntt_plan_t plan) {
  if (check_plan(plan) != NTT_OK) return -1;
  return plan->tuned ? 1 : 0;
}

// Kernels of the transform proper (without the natural-order permutation).
static uint32_t core_passes(ntt_plan_t plan) {
  if (plan->stage_path()) return nttk::stage_group_count(plan->logN, plan->log2_radix);
  return (plan->logN1 && plan->kernel_path != NTT_PATH_FUSED) ? 2u : 1u;
}

uint32_t ntt_plan_num_passes(ntt_plan_t plan) {
  if (check_plan(plan) != NTT_OK) return 0u;
  return core_passes(plan) + (plan->order == NTT_ORDER_NATURAL ? 1u : 0u);
}

static ntt_status run_pass(ntt_plan_t plan, uint64_t* d_data, uint32_t n_polys, uint32_t pass, void* stream,
                           bool inverse) {
  try {
    ntt_status s = check_data(plan, d_data, n_polys);
    if (s != NTT_OK) return s;
    if (pass >= ntt_plan_num_passes(plan)) return fail(NTT_ERR_ARG, "pass index out of range");
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
    const PassArgs a = plan->args(d_data, n_polys, inverse);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    // natural-order plans: the permutation is the last forward pass and the first inverse pass
    if (plan->order == NTT_ORDER_NATURAL) {
      const uint32_t perm_pass = inverse ? 0u : core_passes(plan);
      if (pass == perm_pass) {
        e = nttk::launch_brv_permute(a, st);
        return e == hipSuccess ? NTT_OK : hip_fail(e, "pass launch");
      }
      if (inverse) --pass;
    }
    if (plan->kernel_path == NTT_PATH_FUSED) {
      if (!plan->fused_for(n_polys)) return fail(NTT_ERR_ARG, "batch too large for the fused path's counters");
      e = launch_fused(plan, d_data, n_polys, inverse, st);
    } else if (plan->stage_path()) {
      e = nttk::launch_stage_group(a, plan->log2_radix, inverse, pass, st);
    } else {
      e = inverse ? nttk::launch_inverse_pass(a, plan->active_ot(), (int)pass, st)
                  : nttk::launch_forward_pass(a, plan->active_ot(), (int)pass, st);
    }
    return e == hipSuccess ? NTT_OK : hip_fail(e, "pass launch");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in a pass launch");
  }
}

ntt_status ntt_forward_pass(ntt_plan_t plan, uint64_t* d_data, uint32_t n_polys, uint32_t pass, void* stream) {
  return run_pass(plan, d_data, n_polys, pass, stream, false);
}

ntt_status ntt_inverse_pass(ntt_plan_t plan, uint64_t* d_data, uint32_t n_polys, uint32_t pass, void* stream) {
  return run_pass(plan, d_data, n_polys, pass, stream, true);
}

ntt_status ntt_inverse(ntt_plan_t plan, uint64_t* d_data, uint32_t n_polys, void* stream) {
  try {
    ntt_status s = check_data(plan, d_data, n_polys);
    if (s != NTT_OK) return s;
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
    const hipError_t e = transform(plan, d_data, n_polys, true, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? NTT_OK : hip_fail(e, "ntt_inverse launch");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_inverse");
  }
}

ntt_status ntt_device_copy(void* d_dst, const void* d_src, size_t bytes, void* stream) {
  try {
    if (bytes == 0) return NTT_OK;
    if (!d_dst || !d_src) return fail(NTT_ERR_ARG, "null buffer");
    if (((uintptr_t)d_dst | (uintptr_t)d_src) % 16 != 0) return fail(NTT_ERR_ARG, "buffers must be 16-byte aligned");
    if (bytes % 16 != 0 || bytes >= ((size_t)1 << 35)) return fail(NTT_ERR_ARG, "bytes must be a multiple of 16 below 2^35");
    const uintptr_t a = (uintptr_t)d_dst, b = (uintptr_t)d_src;
    if (a < b + bytes && b < a + bytes) return fail(NTT_ERR_ARG, "buffers overlap");
    const hipError_t e = nttk::launch_copy16(d_src, d_dst, bytes / 16, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? NTT_OK : hip_fail(e, "ntt_device_copy launch");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_device_copy");
  }
}

ntt_status ntt_pointwise_mul(ntt_plan_t plan, const uint64_t* d_a, const uint64_t* d_b, uint64_t* d_c,
                             uint32_t n_polys, void* stream) {
  try {
    ntt_status s;
    if ((s = check_data(plan, d_a, n_polys)) != NTT_OK || (s = check_data(plan, d_b, n_polys)) != NTT_OK ||
        (s = check_data(plan, d_c, n_polys)) != NTT_OK)
      return s;
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
    const uint64_t n = (uint64_t)n_polys * plan->L * plan->N;
    const hipError_t e = nttk::launch_pointwise(d_a, d_b, d_c, plan->d_q, plan->d_mu, plan->d_bits, n, plan->logN,
                                                plan->L, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? NTT_OK : hip_fail(e, "ntt_pointwise_mul launch");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_pointwise_mul");
  }
}

ntt_status ntt_polymul_negacyclic(ntt_plan_t plan, const uint64_t* d_a, const uint64_t* d_b, uint64_t* d_c,
                                  uint32_t n_polys, void* stream) {
  try {
    ntt_status s = check_product(plan, d_a, d_b, d_c, n_polys);
    if (s != NTT_OK) return s;
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t bytes = (size_t)n_polys * plan->L * plan->N * sizeof(uint64_t);

    ntt_plan_s::StreamScratch* sc = plan->scratch_for(st);
    std::lock_guard<std::mutex> lk(sc->mu);
    hipError_t e;
    if (!sc->ev && (e = hipEventCreateWithFlags(&sc->ev, hipEventDisableTiming)) != hipSuccess) {
      sc->ev = nullptr;
      return hip_fail(e, "hipEventCreate");
    }
    if (sc->bytes < bytes) {
      // the old buffer may still feed the last product enqueued on this stream
      if (sc->pending && (e = hipEventSynchronize(sc->ev)) != hipSuccess) return hip_fail(e, "waiting for scratch");
      if (sc->buf) (void)hipFree(sc->buf);
      sc->buf = nullptr;
      sc->bytes = 0;
      sc->pending = false;
      if ((e = hipMalloc(reinterpret_cast<void**>(&sc->buf), bytes)) != hipSuccess)
        return e == hipErrorOutOfMemory ? fail(NTT_ERR_NOMEM, "scratch allocation failed")
                                        : hip_fail(e, "scratch allocation");
      sc->bytes = bytes;
    }
    if ((e = polymul_enqueue(plan, d_a, d_b, d_c, n_polys, sc->buf, st)) != hipSuccess)
      return hip_fail(e, "ntt_polymul_negacyclic launch");
    if ((e = hipEventRecord(sc->ev, st)) != hipSuccess) return hip_fail(e, "recording scratch event");
    sc->pending = true;
    return NTT_OK;
  } catch (const std::bad_alloc&) {
    return fail(NTT_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_polymul_negacyclic");
  }
}

// ---------------------------------------------------------------- product without allocation
// For callers that cannot allocate device memory (graph capture, serving loops): NTT(b) goes
// to a fixed device array instead of a plan-owned buffer.  Each device that loads the library
// holds its own copy of the array until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory, so the array's device address is looked up once per
// device (scratch_address) and only that address is ever passed on.
static constexpr size_t kNoAllocScratchWords = (size_t)1 << 23;   // 64 MiB
static __device__ __align__(256) uint64_t scratch[kNoAllocScratchWords];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint64_t* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on `dev`, which must be the current device.
static ntt_status scratch_address(int dev, uint64_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(NTT_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<uint64_t*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return NTT_OK;
}

uint64_t ntt_polymul_noalloc_max_words(void) { return kNoAllocScratchWords; }

ntt_status ntt_polymul_negacyclic_noalloc(ntt_plan_t plan, const uint64_t* d_a, const uint64_t* d_b, uint64_t* d_c,
                                          uint32_t n_polys, void* stream) {
  try {
    ntt_status s = check_product(plan, d_a, d_b, d_c, n_polys);
    if (s != NTT_OK) return s;
    const uint64_t words = (uint64_t)n_polys * plan->L * plan->N;
    if (words > kNoAllocScratchWords)
      return fail(NTT_ERR_ARG, "n_polys*L*N = " + std::to_string(words) + " exceeds the no-allocation limit of " +
                                   std::to_string(kNoAllocScratchWords) + " residues");
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
    uint64_t* tmp = nullptr;
    if ((s = scratch_address(plan->device, &tmp)) != NTT_OK) return s;
    const hipError_t e = polymul_enqueue(plan, d_a, d_b, d_c, n_polys, tmp, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? NTT_OK : hip_fail(e, "ntt_polymul_negacyclic_noalloc launch");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_polymul_negacyclic_noalloc");
  }
}

ntt_status ntt_batch_create(ntt_batch_t* out, const ntt_job* jobs, uint32_t n_jobs) {
  try {
    if (!out) return fail(NTT_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!jobs || n_jobs == 0) return fail(NTT_ERR_ARG, "jobs must be a non-empty array");
    if (!jobs[0].plan) return fail(NTT_ERR_ARG, "job 0: NULL plan");
    DeviceGuard g(jobs[0].plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plans' device");
    std::unique_ptr<ntt_batch_s> b(new (std::nothrow) ntt_batch_s());
    if (!b) return fail(NTT_ERR_NOMEM, "host allocation failed");
    b->device = jobs[0].plan->device;
    std::vector<nttk::VecDesc> desc;
    ntt_status s = plan_batch(b.get(), jobs, n_jobs, desc);
    if (s != NTT_OK) return s;
    hipError_t e;
    if ((e = hipEventCreateWithFlags(&b->used, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "hipEventCreate");
    if ((s = upload_batch(b.get(), desc, nullptr)) != NTT_OK) return s;
    if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return hip_fail(e, "uploading batch descriptors");
    *out = b.release();
    return NTT_OK;
  } catch (const std::bad_alloc&) {
    return fail(NTT_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_batch_create");
  }
}

ntt_status ntt_batch_assign(ntt_batch_t b, const ntt_job* jobs, uint32_t n_jobs, void* stream) {
  try {
    if (!b) return fail(NTT_ERR_ARG, "batch is NULL");
    DeviceGuard g(b->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the batch's device");
    std::vector<nttk::VecDesc> desc;
    ntt_status s = plan_batch(b, jobs, n_jobs, desc);
    if (s == NTT_OK) s = upload_batch(b, desc, static_cast<hipStream_t>(stream));
    if (s != NTT_OK) {   // leave no job whose descriptors may be missing
      b->jobs.clear();
      b->groups.clear();
      b->drop_graph();
      b->hold({});
    }
    return s;
  } catch (const std::bad_alloc&) {
    return fail(NTT_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_batch_assign");
  }
}

ntt_status ntt_batch_run(ntt_batch_t b, int32_t mode, void* stream) {
  try {
    if (!b) return fail(NTT_ERR_ARG, "batch is NULL");
    DeviceGuard g(b->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the batch's device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (mode < NTT_BATCH_PLAIN || mode > NTT_BATCH_GRAPH_BRANCHED) return fail(NTT_ERR_ARG, "unknown batch mode");
    if (b->jobs.empty()) return NTT_OK;   // emptied by a failed assign
    if (mode == NTT_BATCH_PLAIN) {
      for (const ntt_job& job : b->jobs) {
        const ntt_plan_t pl = job.plan;
        const uint32_t lim = job.n_limbs ? job.n_limbs : pl->L;
        if ((job.op & NTT_OP_FORWARD) && (e = transform(pl, job.d_data, job.n_polys, false, st, job.n_limbs)))
          break;
        if (job.op & NTT_OP_MULKEY) {
          const uint64_t per = (uint64_t)lim * pl->N;
          for (uint32_t p = 0; p < job.n_polys && e == hipSuccess; ++p)
            e = nttk::launch_pointwise(job.d_data + p * per, job.d_key, job.d_data + p * per, pl->d_q, pl->d_mu,
                                       pl->d_bits, per, pl->logN, lim, st);
          if (e != hipSuccess) break;
        }
        if ((job.op & NTT_OP_INVERSE) && (e = transform(pl, job.d_data, job.n_polys, true, st, job.n_limbs)))
          break;
      }
    } else if (mode == NTT_BATCH_GROUPED) {
      e = b->grouped(st);
    } else if (mode == NTT_BATCH_GRAPH) {
      if (!b->exec) {
        // the private capture stream lives as long as the batch: reassigning the jobs drops
        // the graph but keeps the stream
        if (!b->capture_stream &&
            (e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking)) != hipSuccess) {
          b->capture_stream = nullptr;
          return hip_fail(e, "creating the capture stream");
        }
        b->drop_graph();
        if ((e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
          return hip_fail(e, "hipStreamBeginCapture");
        const hipError_t le = b->grouped(b->capture_stream);
        e = hipStreamEndCapture(b->capture_stream, &b->graph);
        if (le != hipSuccess || e != hipSuccess) {
          b->drop_graph();   // a partial graph is never kept or replayed
          return hip_fail(le != hipSuccess ? le : e, le != hipSuccess ? "capturing the batch" : "hipStreamEndCapture");
        }
        if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) {
          b->exec = nullptr;
          b->drop_graph();
          return hip_fail(e, "hipGraphInstantiate");
        }
      }
      e = hipGraphLaunch(b->exec, st);
    } else if (mode == NTT_BATCH_GRAPH_BRANCHED) {
      if (!b->exec_br) {
        if (!b->capture_stream &&
            (e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking)) != hipSuccess) {
          b->capture_stream = nullptr;
          return hip_fail(e, "creating the capture stream");
        }
        if (b->graph_br) (void)hipGraphDestroy(b->graph_br);
        b->graph_br = nullptr;
        if ((e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
          return hip_fail(e, "hipStreamBeginCapture");
        const hipError_t le = b->branched(b->capture_stream);
        e = hipStreamEndCapture(b->capture_stream, &b->graph_br);
        if (le != hipSuccess || e != hipSuccess) {
          if (b->graph_br) (void)hipGraphDestroy(b->graph_br);
          b->graph_br = nullptr;
          return hip_fail(le != hipSuccess ? le : e, le != hipSuccess ? "capturing the batch" : "hipStreamEndCapture");
        }
        if ((e = hipGraphInstantiate(&b->exec_br, b->graph_br, nullptr, nullptr, 0)) != hipSuccess) {
          b->exec_br = nullptr;
          (void)hipGraphDestroy(b->graph_br);
          b->graph_br = nullptr;
          return hip_fail(e, "hipGraphInstantiate");
        }
      }
      e = hipGraphLaunch(b->exec_br, st);
    } else {
      return fail(NTT_ERR_ARG, "unknown batch mode");
    }
    if (e == hipSuccess && (e = hipEventRecord(b->used, st)) == hipSuccess) b->used_pending = true;
    return e == hipSuccess ? NTT_OK : hip_fail(e, "ntt_batch_run");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_batch_run");
  }
}

ntt_status ntt_batch_destroy(ntt_batch_t b) {
  try {
    if (!b) return NTT_OK;
    DeviceGuard g(b->device);
    delete b;
    return NTT_OK;
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_batch_destroy");
  }
}

// ---------------------------------------------------------------- 32-bit words

ntt_status ntt_forward_u32(ntt_plan_t plan, uint32_t* d_data, uint32_t n_polys, void* stream) {
  try {
    if (ntt_status s = check_data_words(plan, d_data, n_polys, 32)) return s;
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
    const hipError_t e = nttk::launch_transform32(d_data, plan->d_tw32_fwd, plan->d_scale32, plan->d_q32,
                                                  (uint64_t)n_polys * plan->L, plan->L, plan->logN, plan->logN1, false,
                                                  static_cast<hipStream_t>(stream));
    return e == hipSuccess ? NTT_OK : hip_fail(e, "ntt_forward_u32 launch");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_forward_u32");
  }
}

ntt_status ntt_inverse_u32(ntt_plan_t plan, uint32_t* d_data, uint32_t n_polys, void* stream) {
  try {
    if (ntt_status s = check_data_words(plan, d_data, n_polys, 32)) return s;
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
    const hipError_t e = nttk::launch_transform32(d_data, plan->d_tw32_inv, plan->d_scale32, plan->d_q32,
                                                  (uint64_t)n_polys * plan->L, plan->L, plan->logN, plan->logN1, true,
                                                  static_cast<hipStream_t>(stream));
    return e == hipSuccess ? NTT_OK : hip_fail(e, "ntt_inverse_u32 launch");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_inverse_u32");
  }
}

ntt_status ntt_pointwise_mul_u32(ntt_plan_t plan, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_c,
                                 uint32_t n_polys, void* stream) {
  try {
    ntt_status s;
    if ((s = check_data_words(plan, d_a, n_polys, 32)) || (s = check_data_words(plan, d_b, n_polys, 32)) ||
        (s = check_data_words(plan, d_c, n_polys, 32)))
      return s;
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
    const hipError_t e = nttk::launch_pointwise32(d_a, d_b, d_c, plan->d_q32, plan->d_mu64,
                                                  (uint64_t)n_polys * plan->L * plan->N, plan->logN, plan->L,
                                                  static_cast<hipStream_t>(stream));
    return e == hipSuccess ? NTT_OK : hip_fail(e, "ntt_pointwise_mul_u32 launch");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_pointwise_mul_u32");
  }
}

ntt_status ntt_polymul_negacyclic_u32(ntt_plan_t plan, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_c,
                                      uint32_t n_polys, void* stream) {
  try {
    ntt_status s;
    if ((s = check_data_words(plan, d_a, n_polys, 32)) || (s = check_data_words(plan, d_b, n_polys, 32)) ||
        (s = check_data_words(plan, d_c, n_polys, 32)))
      return s;
    if (d_c == d_b) return fail(NTT_ERR_ARG, "d_c must not alias d_b");
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t bytes = (size_t)n_polys * plan->L * plan->N * sizeof(uint32_t);
    ntt_plan_s::StreamScratch* sc = plan->scratch_for(st);
    std::lock_guard<std::mutex> lk(sc->mu);
    hipError_t e;
    if (!sc->ev && (e = hipEventCreateWithFlags(&sc->ev, hipEventDisableTiming)) != hipSuccess) {
      sc->ev = nullptr;
      return hip_fail(e, "hipEventCreate");
    }
    if (sc->bytes < bytes) {
      if (sc->pending && (e = hipEventSynchronize(sc->ev)) != hipSuccess) return hip_fail(e, "waiting for scratch");
      if (sc->buf) (void)hipFree(sc->buf);
      sc->buf = nullptr;
      sc->bytes = 0;
      sc->pending = false;
      if ((e = hipMalloc(reinterpret_cast<void**>(&sc->buf), bytes)) != hipSuccess)
        return e == hipErrorOutOfMemory ? fail(NTT_ERR_NOMEM, "scratch allocation failed")
                                        : hip_fail(e, "scratch allocation");
      sc->bytes = bytes;
    }
    uint32_t* tmp = reinterpret_cast<uint32_t*>(sc->buf);
    const uint64_t n_vec = (uint64_t)n_polys * plan->L;
    if ((d_c != d_a && (e = hipMemcpyAsync(d_c, d_a, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) ||
        (e = hipMemcpyAsync(tmp, d_b, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
        (e = nttk::launch_transform32(d_c, plan->d_tw32_fwd, plan->d_scale32, plan->d_q32, n_vec, plan->L, plan->logN,
                                      plan->logN1, false, st)) != hipSuccess ||
        (e = nttk::launch_transform32(tmp, plan->d_tw32_fwd, plan->d_scale32, plan->d_q32, n_vec, plan->L, plan->logN,
                                      plan->logN1, false, st)) != hipSuccess ||
        (e = nttk::launch_pointwise32(d_c, tmp, d_c, plan->d_q32, plan->d_mu64, n_vec * plan->N, plan->logN, plan->L,
                                      st)) != hipSuccess ||
        (e = nttk::launch_transform32(d_c, plan->d_tw32_inv, plan->d_scale32, plan->d_q32, n_vec, plan->L, plan->logN,
                                      plan->logN1, true, st)) != hipSuccess)
      return hip_fail(e, "ntt_polymul_negacyclic_u32 launch");
    if ((e = hipEventRecord(sc->ev, st)) != hipSuccess) return hip_fail(e, "recording scratch event");
    sc->pending = true;
    return NTT_OK;
  } catch (const std::bad_alloc&) {
    return fail(NTT_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_polymul_negacyclic_u32");
  }
}

int32_t ntt_plan_word_bits(ntt_plan_t plan) {
  if (check_plan(plan) != NTT_OK) return -1;
  return plan->word_bits;
}

// ---------------------------------------------------------------- RNS <-> integers

static constexpr uint32_t kCrtMaxLimbs = 64;   // reconstruction keeps L words per lane in LDS (32 KB)

// Build the conversion tables of a 64-bit plan and upload them (once).
static ntt_status crt_prepare(ntt_plan_t plan) {
  std::lock_guard<std::mutex> lk(plan->crt.mu);
  if (plan->crt.ready) return NTT_OK;
  const nttc::CrtTables t = nttc::crt_tables(plan->primes);
  std::vector<Tw> pow2(t.pow2.size()), inv(t.L);
  for (uint32_t l = 0; l < t.L; ++l) {
    const uint64_t q = plan->primes[l];
    for (uint32_t w = 0; w < nttc::kCrtMaxInWords; ++w) {
      const uint64_t c = t.pow2[(size_t)l * nttc::kCrtMaxInWords + w];
      pow2[(size_t)l * nttc::kCrtMaxInWords + w] = Tw{c, nttp::shoup_companion(c, q)};
    }
    inv[l] = Tw{t.inv[l], nttp::shoup_companion(t.inv[l], q)};
  }
  DeviceGuard g(plan->device);
  if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
  hipError_t e;
  if ((e = upload(&plan->crt.pow2, pow2)) != hipSuccess || (e = upload(&plan->crt.inv, inv)) != hipSuccess ||
      (e = upload(&plan->crt.M, t.M)) != hipSuccess || (e = upload(&plan->crt.kQ, t.kQ)) != hipSuccess) {
    if (e == hipErrorOutOfMemory) return fail(NTT_ERR_NOMEM, "device allocation of conversion tables failed");
    return hip_fail(e, "uploading conversion tables");
  }
  plan->crt.W = t.W;
  plan->crt.ready = true;
  return NTT_OK;
}

uint32_t ntt_crt_words(ntt_plan_t plan) {
  try {
    if (check_plan(plan) != NTT_OK || plan->word_bits != 64) return 0;
    if (crt_prepare(plan) != NTT_OK) return 0;
    return plan->crt.W;
  } catch (...) {
    return 0;
  }
}

ntt_status ntt_rns_decompose(ntt_plan_t plan, const uint64_t* d_words, uint32_t n_words, uint64_t* d_res,
                             uint32_t n_polys, void* stream) {
  try {
    ntt_status s;
    if ((s = check_data(plan, d_words, n_polys)) || (s = check_data(plan, d_res, n_polys))) return s;
    if (n_words == 0 || n_words > nttc::kCrtMaxInWords)
      return fail(NTT_ERR_ARG, "n_words must be 1.." + std::to_string(nttc::kCrtMaxInWords));
    if ((s = crt_prepare(plan))) return s;
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
    const hipError_t e = nttk::launch_rns_decompose(d_words, n_words, d_res, n_polys, plan->logN, plan->L,
                                                    plan->crt.pow2, nttc::kCrtMaxInWords, plan->d_q,
                                                    static_cast<hipStream_t>(stream));
    return e == hipSuccess ? NTT_OK : hip_fail(e, "ntt_rns_decompose launch");
  } catch (const std::bad_alloc&) {
    return fail(NTT_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_rns_decompose");
  }
}

ntt_status ntt_crt_reconstruct(ntt_plan_t plan, const uint64_t* d_res, uint64_t* d_words, uint32_t n_polys,
                               void* stream) {
  try {
    ntt_status s;
    if ((s = check_data(plan, d_res, n_polys)) || (s = check_data(plan, d_words, n_polys))) return s;
    if (plan->L > kCrtMaxLimbs)
      return fail(NTT_ERR_UNSUPPORTED, "reconstruction takes at most " + std::to_string(kCrtMaxLimbs) + " primes");
    if (d_res == d_words) return fail(NTT_ERR_ARG, "d_words must not alias d_res");
    if ((s = crt_prepare(plan))) return s;
    DeviceGuard g(plan->device);
    if (!g.ok) return fail(NTT_ERR_HIP, "cannot select the plan's device");
    const hipError_t e = nttk::launch_crt_reconstruct(d_res, d_words, n_polys, plan->logN, plan->L, plan->crt.W,
                                                      plan->crt.inv, plan->crt.M, plan->crt.kQ, plan->d_q,
                                                      static_cast<hipStream_t>(stream));
    return e == hipSuccess ? NTT_OK : hip_fail(e, "ntt_crt_reconstruct launch");
  } catch (const std::bad_alloc&) {
    return fail(NTT_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(NTT_ERR_ARG, "unexpected failure in ntt_crt_reconstruct");
  }
}

const char* ntt_status_string(ntt_status s) {
  switch (s) {
    case NTT_OK: return "NTT_OK";
    case NTT_ERR_ARG: return "NTT_ERR_ARG";
    case NTT_ERR_N: return "NTT_ERR_N";
    case NTT_ERR_PRIME: return "NTT_ERR_PRIME";
    case NTT_ERR_NOMEM: return "NTT_ERR_NOMEM";
    case NTT_ERR_HIP: return "NTT_ERR_HIP";
    case NTT_ERR_UNSUPPORTED: return "NTT_ERR_UNSUPPORTED";
  }
  return "NTT_ERR_UNKNOWN";
}

const char* ntt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
