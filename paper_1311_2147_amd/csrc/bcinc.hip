// libbcinc as one translation unit: kernels first, then the C ABI.
#include "bc_kernels.hip"
#include "bc_host.hip"
