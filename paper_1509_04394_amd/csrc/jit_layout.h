// How a generated kernel lays out its work (host code, shared by the
// generator and the planner): the cells per thread of each window stage and
// the LDS row pitch of the group's buffers.
#pragma once

#include <vector>

#include "generic.h"

namespace fz {

// How each window stage of a group is computed: cells per thread across (gq)
// and down (gr), and the halo left around its output region (ohx, ohy).
struct WinStep {
    int i, j;  // the window stage and the stage after its trailing point stages
    bool last;
    int ohx, ohy, gq, gr;
};

std::vector<WinStep> win_steps(const GStage* st, int n, int TW, int TH, int HX, int HY);


}  // namespace fz
