// One (storage type, block width) slice of the scan kernel's instantiations.
// The build compiles this file once per pair, with ADS_SCAN_DT set to an
// ads_dtype and ADS_SCAN_DD to a block width, so the many template
// instantiations compile in parallel.
#include "scan_kernel.h"

#ifndef ADS_SCAN_DT
#error "ADS_SCAN_DT (storage type) must be defined"
#endif
#ifndef ADS_SCAN_DD
#error "ADS_SCAN_DD (block width) must be defined"
#endif

namespace ads {
template hipError_t launch_scan_q<ADS_SCAN_DT, ADS_SCAN_DD>(const ScanArgs &, int, int, bool, bool, hipStream_t);
}  // namespace ads
