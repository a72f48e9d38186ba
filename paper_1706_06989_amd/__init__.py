"""MI355X-native angular-momentum-conserving Cartesian FMM (Marcello 2017).

The solver is the HIP library ``libamfmm_hip.so`` behind the C ABI of
``include/amfmm.h``; ``paper_1706_06989_amd.amfmm`` is its thin Python binding
(argument marshalling only).  ``paper_1706_06989_amd.workloads`` draws seeded
synthetic inputs.  Importing the package loads nothing native.
"""
