// select.h -- which vertex slot i of a CC/SSSP exchange launch runs
// (selection of the active vertices, Section 4.3.1).  Plain C++ behind the
// HIP qualifiers: the library compiles it as device code, and a CPU test
// builds the same function with the qualifiers defined empty and checks it
// under the compiler's warnings and sanitizers.
#pragma once

#include <stdint.h>

namespace ipg {

// Which vertices run compute in a launch.
enum : int {
  kSendAll = 0,     // superstep 0 of CC: every vertex broadcasts its id
  kSendSource = 1,  // superstep 0 of SSSP: the source broadcasts
  kStepList = 2,    // s >= 1, active vertices given as a list
  kStepDense = 3    // s >= 1, active vertices = non-empty mailboxes (sweep all N)
};

// Segments of the frontier list (one per counter slot).
constexpr uint32_t kListSegs = 64;

struct Active {
  int phase;
  uint32_t count;           // list length, or N for the dense and send-all phases
  const uint32_t* list;     // the list, in kListSegs segments of `seg` entries
  const uint32_t* pre;      // [kListSegs + 1] prefix of the segments' lengths
  uint32_t seg;
  uint32_t source;
};

// Vertex of slot i < act.count of a launch.  List entry i lies in the
// segment k with s_pre[k] <= i < s_pre[k + 1] (s_pre: the prefix of the
// segments' lengths, s_pre[0] = 0, s_pre[kListSegs] = act.count).  Every
// path assigns every value it uses: the segment search always starts at 0,
// the list is read only in the list phase, and the send-source phase
// returns the source whatever the slot.
__host__ __device__ __forceinline__ uint32_t active_vertex(const Active& act, const uint32_t* s_pre, uint64_t i) {
  const uint32_t id = static_cast<uint32_t>(i);
  const bool listed = act.phase == kStepList;  // uniform over the grid
  uint32_t lo = 0;
  if (listed) {
    uint32_t hi = kListSegs - 1;  // the last k with s_pre[k] <= i
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (s_pre[mid] <= id) lo = mid;
      else hi = mid - 1;
    }
  }
  const uint64_t li = listed ? static_cast<uint64_t>(lo) * act.seg + (id - s_pre[lo]) : 0;
  const uint32_t from_list = listed ? act.list[li] : id;
  return act.phase == kSendSource ? act.source : from_list;
}

}  // namespace ipg
