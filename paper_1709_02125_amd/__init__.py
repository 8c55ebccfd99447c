"""Out-of-core tiled stencil loop chains on MI355X (gfx950).

The HIP library (libooc.so, C ABI in include/ooc.h) holds the whole path:
lazy loop queue, dependency analysis and skewed tiling, slot memory manager,
three-stream pipeline and the stencil kernels.  `ooc` is its ctypes binding;
`hydro2d` drives the 2D hydro proxy through it; `inputs` holds the seeded
synthetic inputs.  Import of the binding fails if the library is not built."""
