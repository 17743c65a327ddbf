// Host check of the plan lifetime rules (compiled with g++ by the test suite).  Random
// sequences of plan creation, batch assignment, batch destruction and plan destruction drive
// the same reference-count helpers the library uses; a reference model says when each plan
// may be finalised.  Checked after every operation:
//   * a plan is finalised exactly once, and only when its creator has destroyed it and no
//     live batch names it;
//   * a plan named by a live batch is never finalised, even after ntt_plan_destroy;
//   * destroying a plan twice is reported and changes nothing.
#include <cstdio>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "plan_life.hpp"

struct FakePlan {
  nttl::RefCount rc;
  int id;
  bool finalised = false;
};

static long failures = 0;
static void fail(const char* what, int id) {
  if (failures++ < 10) std::printf("FAIL %s (plan %d)\n", what, id);
}

int main() {
  std::mt19937 g(2012);
  for (int trial = 0; trial < 2000; ++trial) {
    std::vector<FakePlan*> plans;                 // every plan ever created in this trial
    std::set<FakePlan*> owned;                    // created and not yet destroyed by the creator
    std::map<int, std::vector<FakePlan*>> batches;  // live batches -> distinct plans they hold
    int next_batch = 0;
    auto rc = [](FakePlan* p) -> nttl::RefCount& { return p->rc; };
    auto finalise = [&](const std::vector<FakePlan*>& last) {
      for (FakePlan* p : last) {
        if (p->finalised) fail("finalised twice", p->id);
        p->finalised = true;
      }
    };
    for (int step = 0; step < 60; ++step) {
      const int op = (int)(g() % 5);
      if (op == 0 || plans.empty()) {             // ntt_plan_create
        FakePlan* p = new FakePlan();
        p->id = (int)plans.size();
        plans.push_back(p);
        owned.insert(p);
      } else if (op == 1) {                       // ntt_batch_create / ntt_batch_assign
        std::vector<FakePlan*> jobs;
        const int n = 1 + (int)(g() % 6);
        for (int j = 0; j < n; ++j) {
          FakePlan* p = plans[g() % plans.size()];
          if (p->finalised) continue;             // callers only name live plans
          if (!owned.count(p)) {
            bool held = false;                    // ... a destroyed plan is reachable only through a batch
            for (auto& b : batches)
              for (FakePlan* q : b.second) held = held || q == p;
            if (!held) continue;
          }
          jobs.push_back(p);
        }
        const bool reuse = !batches.empty() && (g() & 1);
        const int id = reuse ? std::next(batches.begin(), g() % batches.size())->first : next_batch++;
        std::vector<FakePlan*> prev = batches.count(id) ? batches[id] : std::vector<FakePlan*>{};
        std::vector<FakePlan*> next = nttl::distinct(jobs);
        finalise(nttl::rehold(prev, next, rc));
        batches[id] = next;
      } else if (op == 2 && !batches.empty()) {   // ntt_batch_destroy
        auto it = std::next(batches.begin(), g() % batches.size());
        finalise(nttl::rehold(it->second, std::vector<FakePlan*>{}, rc));
        batches.erase(it);
      } else {                                    // ntt_plan_destroy (possibly a second time)
        FakePlan* p = plans[g() % plans.size()];
        if (p->finalised) continue;               // a finalised plan is gone: callers may not name it
        const bool was_owned = owned.count(p) != 0;
        const auto r = p->rc.release_owner();
        if (!was_owned && r != nttl::RefCount::kAlreadyGone) fail("second destroy not reported", p->id);
        if (was_owned && r == nttl::RefCount::kAlreadyGone) fail("first destroy reported as second", p->id);
        owned.erase(p);
        if (r == nttl::RefCount::kLast) finalise({p});
      }
      // the model: finalised exactly when not owned and held by no live batch
      for (FakePlan* p : plans) {
        bool held = owned.count(p) != 0;
        for (auto& b : batches)
          for (FakePlan* q : b.second) held = held || q == p;
        if (held && p->finalised) fail("finalised while held", p->id);
        if (!held && !p->finalised) fail("not finalised after its last holder let go", p->id);
      }
    }
    for (FakePlan* p : plans) delete p;
  }
  std::printf("%ld failures\n", failures);
  return failures != 0;
}
