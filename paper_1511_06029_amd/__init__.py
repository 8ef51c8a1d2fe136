"""QTT matrix apply and refined solve on MI355X (gfx950).

The compute path lives in the HIP library ``libqtt.so`` (``csrc/``); the
binding in :mod:`paper_1511_06029_amd.qtt` only marshals arguments to it.
Importing this package does not load the library; importing ``.qtt`` does,
and fails loudly if it has not been built.
"""
