"""FP64 CPU oracle for batched r-cell MD.

TEST INFRASTRUCTURE ONLY.  Imported by the tests, the smoke check and the benchmark's CPU
baseline leg; the GPU library never imports, links or runs anything here, and nothing here
imports the GPU library.  `oracle.core` wraps the plain C implementation (rcell_oracle.c);
`oracle.brute` is an independent numpy O(N^2) twin used to check it on tiny cells;
`oracle.surrogate` is the FP64 numpy reference of the stress surrogate network.
"""
