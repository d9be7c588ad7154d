"""MI355X (gfx950) efficient permutation two-sample test (energy distance / MMD).

The numerical path lives in the HIP library ``libetest.so`` (C ABI in
``include/etest.h``); ``api`` marshals arguments to it.  Nothing is loaded at
import time, so ``inputs`` can be imported on a machine without a GPU.
"""

__all__ = ["api", "inputs", "build"]
