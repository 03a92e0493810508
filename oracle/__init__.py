"""CPU oracle for HoSZp (arXiv 2408.11971) -- test infrastructure only.

Imported by the tests, the smoke check and the benchmark's CPU-baseline leg;
never by the GPU library.  See ``hoszp_ref.c`` for the steps and readings.
"""
