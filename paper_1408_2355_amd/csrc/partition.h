// Region adjacency of a partition (partition.cpp).
#pragma once

#include "internal.h"

namespace sp {

// labels [nres][n] caller order (region index per vertex, other values
// ignored); adj [sum m_r^2] host, restart blocks in order, 1 where regions i
// and j of a restart touch across a mesh edge; sides [sum m_r] (nullable):
// neighbours per region.
void region_graph(const Mesh& mesh, int nres, const int* m, const int32_t* labels, uint8_t* adj,
                  int32_t* sides);

}  // namespace sp
