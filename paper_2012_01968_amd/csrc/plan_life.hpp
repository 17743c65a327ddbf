// Lifetime of plans shared between their creator and the batches that name them (host side
// only; no device code, so the host test suite compiles it with g++).
//
// A plan starts with one reference, its creator's.  A batch takes one reference per distinct
// plan among its jobs and drops them when its jobs are replaced or the batch is destroyed.
// ntt_plan_destroy drops the creator's reference (once).  The plan is finalised (its device
// memory freed) by whichever call drops the last reference, so a plan destroyed while a batch
// still names it stays usable by that batch until the batch lets go.
#pragma once
#include <atomic>
#include <vector>

namespace nttl {

struct RefCount {
  std::atomic<int> refs{1};             // the creator's reference
  std::atomic<bool> owner_gone{false};  // the creator has dropped its reference

  void retain() { refs.fetch_add(1, std::memory_order_relaxed); }
  // true when this call dropped the last reference: the caller finalises the object
  bool release() { return refs.fetch_sub(1, std::memory_order_acq_rel) == 1; }

  enum OwnerRelease { kAlreadyGone, kStillHeld, kLast };
  // Drop the creator's reference, at most once.
  OwnerRelease release_owner() {
    bool expected = false;
    if (!owner_gone.compare_exchange_strong(expected, true)) return kAlreadyGone;
    return release() ? kLast : kStillHeld;
  }
};

// The distinct entries of `items`, in first-seen order (a batch names few plans).
template <typename T>
std::vector<T> distinct(const std::vector<T>& items) {
  std::vector<T> out;
  for (const T& x : items) {
    bool seen = false;
    for (const T& y : out) seen = seen || y == x;
    if (!seen) out.push_back(x);
  }
  return out;
}

// Replace a holder's set of references: every entry of `next` is retained before any entry
// of `prev` is released, so an object held by both is never finalised in between.  Returns
// the entries whose last reference this dropped; the caller finalises them.
template <typename T, typename GetRc>
std::vector<T> rehold(const std::vector<T>& prev, const std::vector<T>& next, GetRc rc) {
  for (const T& x : next) rc(x).retain();
  std::vector<T> last;
  for (const T& x : prev)
    if (rc(x).release()) last.push_back(x);
  return last;
}

}  // namespace nttl
