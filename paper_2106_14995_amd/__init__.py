"""MI355X-native batched trust-region Newton (TRON) solves and the component ADMM.

Importing the package loads nothing; the GPU library is opened by
``paper_2106_14995_amd.tron`` on first use.
"""
