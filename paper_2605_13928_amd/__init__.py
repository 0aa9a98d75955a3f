"""MI355X-native exact t-SNE hot path: HIP kernels for gfx950 behind a C ABI.

The compute path is `libtsne_mi355x.so` (built from `csrc/`); `api` marshals
torch tensors into its calls and `autograd` wraps the KL forward/backward.
Importing this package does not load the library; the first API call does,
and fails loudly when it is missing.
"""
__version__ = "0.1.0"
