"""FP64 CPU oracle for DF-SS-FNO-EA-ADC(3).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product library never imports, links or runs
anything here, and nothing here imports the product library.
"""
