"""librepair: MI355X-native data-parallel hot path of GPURepair's repair loop.

Import ``paper_2011_08373_amd.librepair`` for the C-ABI binding (it loads the
HIP library and fails loudly when it is not built) and
``paper_2011_08373_amd.synth`` for seeded synthetic kernel models.
"""
