// Library-internal accessors shared between the C-ABI translation units.
#pragma once

#include "hgmm_dev.h"

struct hgmm_forest_s;

int hgmm_fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int hgmm_forest_size(const hgmm_forest_s* f);
hgmm::TreeDev* hgmm_forest_trees(hgmm_forest_s* f);
hgmm::NodeD* hgmm_forest_nodes(hgmm_forest_s* f);
