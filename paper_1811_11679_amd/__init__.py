"""MI355X-native FCIQMC hot path: HIP kernels behind a C ABI (include/fciqmc.h)."""
