// Host overset assembly of libugks (Sec. 3.1 mesh assembly, Sec. 3.2
// interpolation weights): node classes, cell classes with one buffer layer
// and the fringe beside overset sides, donors and weights.
#pragma once
#include <string>
#include <vector>

namespace ugks {

struct OversetInput {
  int nblock = 0;
  std::vector<int> ni, nj, cell0, bc;  // bc: 4 per block
  const std::vector<double>* xn = nullptr;  // current nodes, blocks concatenated
  const std::vector<double>* yn = nullptr;
  const std::vector<size_t>* node0 = nullptr;
  const std::vector<double>* cx = nullptr;  // cell centroids and areas
  const std::vector<double>* cy = nullptr;
  const std::vector<double>* vol = nullptr;
  const std::vector<signed char>* old_type = nullptr;  // cell kinds before this assembly
};

struct OversetOutput {
  std::vector<signed char> type;  // per cell: 0 hole, 1 field, 2 receptor
  // donor rows: the nrec receptors, then the cells that were holes and are
  // field now (interpolated once, at the start of the next physical step)
  int nrec = 0;
  std::vector<int> rec, ptr, don;
  std::vector<double> w;
};

// returns 0 or a negative UGKS_E_* code with a message; on error `out` is
// left unspecified and nothing should be installed
int overset_build(const OversetInput& in, int wrule, int overlap, OversetOutput& out, std::string& msg);
// the same assembly on the current HIP device (ugks_overset_dev.hip), with
// identical results
int overset_build_device(const OversetInput& in, int wrule, int overlap, OversetOutput& out, std::string& msg);

}  // namespace ugks
