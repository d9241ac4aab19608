"""CPU oracle for the MONC advection path -- test infrastructure only.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never does.
"""
