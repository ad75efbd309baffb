// libbcinc as one translation unit: kernels first (the update path, then the
// state check), then the C ABI.
#include "bc_kernels.hip"
#include "bc_check.hip"
#include "bc_host.hip"
