"""MI355X-native structured-grid weather step (kinematic FV dycore + column physics).

The compute path is the HIP library ``libwx.so`` behind ``include/wx.h``;
``paper_1802_05839_amd.wx`` is its Python binding and
``paper_1802_05839_amd.inputs`` draws seeded synthetic problems.
"""
__all__ = ["inputs", "wx"]
