"""HalftimeHash on MI355X: hand-written HIP kernels behind a C ABI (libhth)."""
