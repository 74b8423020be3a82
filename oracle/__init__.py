"""FP64 CPU oracle of the per-frame deformation solve (test infrastructure only).

Only the test suite, the smoke entry point and the benchmark's CPU-baseline leg may import this
package. The GPU library never imports, links or calls it.
"""
