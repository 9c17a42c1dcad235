"""MI355X-native fast Fourier transform on SO(3) (Kostelec-Rockmore SOFT).

The compute path lives in the HIP library ``libsoft.so`` (C-ABI declared in
``include/soft.h``); ``soft`` is its thin Python binding.  Importing this
package loads nothing; the library is loaded on first use.
"""
__all__ = ["inputs"]
