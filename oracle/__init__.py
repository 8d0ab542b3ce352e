"""FP64 CPU oracle of the block transform -- test infrastructure only.

Only `tests/`, the package smoke check and the benchmark's CPU baseline may
import this package; the GPU library never does.
"""
