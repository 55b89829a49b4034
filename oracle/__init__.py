"""CPU oracle of the kernel-compressed time-fractional stress update.

Test infrastructure only: tests, the smoke check and the benchmark's CPU
baseline may use it; the product library never imports or links it.
"""
