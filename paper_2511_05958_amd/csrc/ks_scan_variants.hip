// One scan-kernel variant (KS_SCAN_VARIANT, an index into ks_host::kVariants)
// for every K class and launch mode: this file is compiled once per variant.
#include <hip/hip_runtime.h>

#include "ks_ctx.hpp"
#include "ks_persist.hpp"

#ifndef KS_SCAN_VARIANT
#error "compile once per variant with -DKS_SCAN_VARIANT=<index>"
#endif

namespace ks_host {

namespace {
constexpr Variant kV = kVariants[KS_SCAN_VARIANT];

template <int KMAX>
ScanKernels kernels_of() {
  return ScanKernels{reinterpret_cast<const void*>(&ks::scan_kernel<KMAX, kV.nt, kV.rb, kV.gm>),
                     reinterpret_cast<const void*>(&ks::scan_persistent<KMAX, kV.nt, kV.rb, kV.gm>),
                     reinterpret_cast<const void*>(&ks::finish_kernel<KMAX, kV.nt, kV.rb, kV.gm>)};
}
}  // namespace

#define KS_TABLE_NAME2(v) scan_table_##v
#define KS_TABLE_NAME(v) KS_TABLE_NAME2(v)

extern const ScanKernels KS_TABLE_NAME(KS_SCAN_VARIANT)[kNumKClasses];
const ScanKernels KS_TABLE_NAME(KS_SCAN_VARIANT)[kNumKClasses] = {kernels_of<64>(),  kernels_of<128>(),
                                                                   kernels_of<256>(), kernels_of<512>(),
                                                                   kernels_of<1024>(), kernels_of<2048>()};

}  // namespace ks_host
