"""Seeded synthetic inputs shared by the GPU path and the test oracle.

This package holds setup code only (TOV background, particle placement, the synthetic EoS
table, workload configurations).  It contains none of the per-step particle-loop arithmetic
and imports neither the GPU package nor the oracle.
"""
