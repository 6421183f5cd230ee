"""Seeded synthetic inputs and workload recipes shared by the tests, the smoke
check and the benchmark.  Holds no transform code of the GPU library or of the
oracle."""
