"""MI355X-native compute point-cloud rasterizer (gfx950 HIP kernels behind a C ABI).

Implements the rendering passes of Schuetz, Kerbl and Wimmer, "Rendering Point
Clouds with Compute Shaders and Vertex Order Optimization" (EGSR 2021): the
64-bit atomicMin closest-point renderer (Sec. 3.1), its early-depth-test and
local deduplication forms (Sec. 3.2-3.4), the two-pass high-quality blend
(Sec. 3.5) and the Morton / shuffled-Morton vertex orders (Sec. 4).

The compiled library ``libpcr.so`` does all the work; ``pcr`` is its ctypes
binding.  Importing the package does not load the library, so that the pure
host modules (``synth``) work without it.
"""

__all__ = ["pcr", "synth"]
