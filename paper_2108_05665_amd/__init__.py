"""MI355X (gfx950) multi-tensor contraction for XEB verification.

Hot path: libxeb.so (hand-written HIP + C++ runtime behind the C ABI in
include/xeb.h).  `xeb` is its ctypes binding; `planner` produces contraction
trees and slice lists on the host.
"""

__all__ = ["xeb", "planner", "build"]
