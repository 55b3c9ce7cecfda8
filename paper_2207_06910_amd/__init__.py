"""MI355X-native Fisher/SNR hot path of the GWFAST method (arXiv:2207.06910)."""
