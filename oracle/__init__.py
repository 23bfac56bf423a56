"""FP64 CPU oracle for Lagrangian RK4 advection -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  It shares no code with the HIP library and never imports it.
"""
