"""MI355X-native space-time multigrid for the eddy-current equation.

Importing the package loads nothing; ``paper_1911_09548_amd.stmg`` is the
ctypes binding of the HIP library and ``paper_1911_09548_amd.inputs`` holds
the seeded synthetic problem generators.
"""
