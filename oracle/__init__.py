"""CPU oracle (test infrastructure only): plain C loops + Python orchestration.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It shares no code with the GPU library.
"""
