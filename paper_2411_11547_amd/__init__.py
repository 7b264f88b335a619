"""MI355X-native Pair-HMM forward algorithm (arXiv 2411.11547) for gfx950.

The arithmetic lives in hand-written HIP kernels behind the C ABI of
``libpairhmm.so`` (declared in ``include/ph.h``).  ``binding`` marshals
arguments to it; ``autograd`` wraps forward/backward as a torch autograd
Function; ``workloads`` generates seeded synthetic inputs.  Importing this
package loads nothing; the library is loaded on first use.
"""
