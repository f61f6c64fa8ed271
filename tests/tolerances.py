"""Parity tolerances of the device paths against the CPU oracle, in one
place (relative, per entry: |y - y*| <= tol |y*|, and exactly 0 where the
oracle gives 0).

F64       1e-12   double vectors and double accumulation
F32C      1e-5    float vectors; row partials in double, reuse chains as
                  TwoSum-compensated float pairs
F32_NAIVE 1e-3    float vectors and float accumulation along reuse chains,
                  interval sums from float prefix sums: an uncompensated
                  comparison mode that does NOT meet the 1e-5 FP32 bar (its
                  error grows with chain depth and with the prefix sums'
                  magnitude; about 2e-5 on the social-like workload)
"""
F64 = 1e-12
F32C = 1e-5
F32_NAIVE = 1e-3
