"""Test infrastructure: the independent CPU oracle for the ziggurat Gaussian path.

Nothing in the product package imports this package. Only the tests, the
smoke check and the CPU-baseline leg of the benchmark use it.
"""
