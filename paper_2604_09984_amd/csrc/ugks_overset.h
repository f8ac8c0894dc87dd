// Host overset assembly of libugks (hole cutting, buffer layer, donors).
#pragma once
#include <string>
#include <vector>

namespace ugks {

struct OversetInput {
  int nblock = 0;
  std::vector<int> ni, nj, cell0, bc;  // bc: 4 per block
  const std::vector<double>* xn = nullptr;
  const std::vector<double>* yn = nullptr;
  const std::vector<size_t>* node0 = nullptr;
};

struct OversetOutput {
  std::vector<signed char> type;  // per cell: 0 hole, 1 field, 2 receptor
  std::vector<int> rec, ptr, don;
  std::vector<double> w;
};

// returns 0 or a negative UGKS_E_* code with a message
int overset_build(const OversetInput& in, int wrule, int overlap, OversetOutput& out, std::string& msg);

}  // namespace ugks
