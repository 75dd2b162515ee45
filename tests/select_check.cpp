// Host check of the push launches' vertex selection (select.h), built with
// g++ -Wall -Wextra -Werror and AddressSanitizer + UndefinedBehaviorSanitizer:
// for random frontier lists cut into kListSegs segments of random lengths
// (every segment fill from 0 to its capacity, empty lists included), every
// slot of every phase must give the expected vertex -- list slot i the i-th
// entry in segment order, a dense or send-all slot its own index, every
// send-source slot the source -- reading only the list's filled entries
// (the list buffer holds exactly the segments' capacity, so a read past it
// trips AddressSanitizer, and a read of an unfilled entry returns a value the
// comparison rejects).  Prints "OK <cases>" or "FAIL <what>".
#define __host__
#define __device__
#define __forceinline__ inline
#include "select.h"

#include <cstdio>
#include <random>
#include <vector>

using namespace ipg;

int main() {
  std::mt19937_64 rng(7);
  uint64_t cases = 0;
  for (int trial = 0; trial < 400; ++trial) {
    const uint32_t seg = 1 + static_cast<uint32_t>(rng() % 97);
    std::vector<uint32_t> len(kListSegs), pre(kListSegs + 1, 0);
    const int shape = trial % 4;  // empty, full, sparse, random
    for (uint32_t k = 0; k < kListSegs; ++k) {
      len[k] = shape == 0 ? 0 : shape == 1 ? seg : shape == 2 ? (rng() % 5 == 0 ? 1 : 0) : static_cast<uint32_t>(rng() % (seg + 1));
      pre[k + 1] = pre[k] + len[k];
    }
    const uint32_t count = pre[kListSegs];
    // the buffer is exactly kListSegs * seg entries; unfilled entries are left uninitialised on purpose
    uint32_t* list = new uint32_t[static_cast<size_t>(kListSegs) * seg];
    std::vector<uint32_t> expect;
    for (uint32_t k = 0; k < kListSegs; ++k)
      for (uint32_t j = 0; j < len[k]; ++j) {
        const uint32_t v = static_cast<uint32_t>(rng() % 1000003);
        list[static_cast<size_t>(k) * seg + j] = v;
        expect.push_back(v);
      }
    for (int phase : {kSendAll, kSendSource, kStepList, kStepDense}) {
      Active act;
      act.phase = phase;
      act.count = phase == kStepList ? count : 1000;
      act.list = list;
      act.pre = pre.data();
      act.seg = seg;
      act.source = 4242;
      for (uint64_t i = 0; i < act.count; ++i) {
        const uint32_t v = active_vertex(act, pre.data(), i);
        const uint32_t want = phase == kStepList ? expect[i] : phase == kSendSource ? 4242u : static_cast<uint32_t>(i);
        if (v != want) {
          std::printf("FAIL phase %d slot %llu: %u, want %u\n", phase, static_cast<unsigned long long>(i), v, want);
          return 1;
        }
        ++cases;
      }
    }
    delete[] list;
  }
  std::printf("OK %llu\n", static_cast<unsigned long long>(cases));
  return 0;
}
