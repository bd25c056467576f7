// Read access to a plan's pair descriptors for the optimisers built on the
// C ABI (not exported).
#pragma once

#include <string>

#include "shoot.h"

// Number of pairs of the plan and a pointer to its descriptors (valid while the
// plan lives); -1 for a NULL plan. *bound: the plan has a workspace.
int shoot_internal_pairs(shoot_plan plan, const shoot_pair** pairs, int* bound);
// Sets the message shoot_last_error returns (this thread).
void shoot_internal_set_error(const char* msg);
// The plan's tuning shape class (shoot_plan_tune_class); "" for NULL.
std::string shoot_internal_tune_class(shoot_plan plan);
// Device the plan was bound on (-1: NULL or unbound); *unfused: SHOOT_UNFUSED.
int shoot_internal_device(shoot_plan plan, int* unfused);
