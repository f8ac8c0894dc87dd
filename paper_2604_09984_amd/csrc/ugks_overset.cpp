// Host overset assembly of libugks.
#include "ugks_overset.h"

#include "ugks.h"

namespace ugks {

int overset_build(const OversetInput& in, int wrule, int overlap, OversetOutput& out, std::string& msg) {
  (void)in; (void)wrule; (void)overlap; (void)out;
  msg = "overset assembly not available";
  return UGKS_E_UNSUPPORTED;
}

}  // namespace ugks
