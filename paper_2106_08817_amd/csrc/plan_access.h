// Read access to a plan's pair descriptors for the optimisers built on the
// C ABI (not exported).
#pragma once

#include "shoot.h"

// Number of pairs of the plan and a pointer to its descriptors (valid while the
// plan lives); -1 for a NULL plan. *bound: the plan has a workspace.
int shoot_internal_pairs(shoot_plan plan, const shoot_pair** pairs, int* bound);
// Sets the message shoot_last_error returns (this thread).
void shoot_internal_set_error(const char* msg);
