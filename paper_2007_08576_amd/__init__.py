"""MI355X-native per-frame deformation solve (Zhou & Jagadeesan, arXiv:2007.08576).

The product is the HIP library under csrc/ behind the C ABI in include/tt.h; `tt` is its thin
ctypes binding. `synth` generates seeded synthetic workloads.
"""
