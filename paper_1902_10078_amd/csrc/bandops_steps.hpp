// bandops_steps.hpp -- the work-item type of every (step, bandwidth, storage).
#pragma once
#include "bandops_driver.hpp"

namespace bo {

// Calls f.template go<Item>() for the item of `step` at bandwidth K and
// storage type T; returns -1 for an unknown step.
template <int K, typename T, class F> int with_item(int step, F &&f) {
  switch (step) {
    case ST_F1_SUM: return f.template go<F1Summary<K, T>>();
    case ST_F1_GCOMP: return f.template go<F1GroupCompose<K>>();
    case ST_F1_GSWEEP: return f.template go<F1GroupSweep<K>>();
    case ST_F1_CSWEEP: return f.template go<F1ChunkSweep<K>>();
    case ST_F1_REP: return f.template go<F1Replay<K, T>>();
    case ST_PC: return f.template go<PcItem<K, T>>();
    case ST_FS_SUM: return f.template go<LinSummary<K, T, PASS_FS>>();
    case ST_FS_REP: return f.template go<LinReplay<K, T, PASS_FS>>();
    case ST_F2_SUM: return f.template go<LinSummary<K, T, PASS_F2>>();
    case ST_F2_REP: return f.template go<LinReplay<K, T, PASS_F2>>();
    case ST_B1_SUM: return f.template go<LinSummary<K, T, PASS_B1>>();
    case ST_B1_REP: return f.template go<LinReplay<K, T, PASS_B1>>();
    case ST_B2_SUM: return f.template go<LinSummary<K, T, PASS_B2>>();
    case ST_B2_REP: return f.template go<LinReplay<K, T, PASS_B2>>();
    case ST_ASC_GCOMP: return f.template go<LinGroupCompose<K, false>>();
    case ST_ASC_GSWEEP: return f.template go<LinGroupSweep<K, false>>();
    case ST_ASC_CSWEEP: return f.template go<LinChunkSweep<K, false>>();
    case ST_DESC_GCOMP: return f.template go<LinGroupCompose<K, true>>();
    case ST_DESC_GSWEEP: return f.template go<LinGroupSweep<K, true>>();
    case ST_DESC_CSWEEP: return f.template go<LinChunkSweep<K, true>>();
    default: return -1;
  }
}

}  // namespace bo
