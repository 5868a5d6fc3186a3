"""MI355X-native per-cycle grid update of a SALE-type r-z impact hydrocode with
perfectly matched layers (Li et al., SALEc-2D).

The compute path is the HIP library ``libsalec`` (C ABI in ``include/salec.h``);
``paper_2403_04267_amd.salec`` is its thin Python binding. Importing this
package loads nothing; the binding loads the library on first use and raises
if it is missing.
"""
__all__ = ["inputs"]
