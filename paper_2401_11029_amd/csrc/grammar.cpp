// grammar.cpp -- parse the grammar text and lower it to strict WCNF.
//
// Definition 1 of the paper allows only x -> t, x -> eps and x -> y z with
// y, z non-terminals; its appendix grammars (Figs. 4b-7b) also put terminals
// in binary right-hand sides and use the unit rule V -> M (Fig. 6b), and the
// grammars taken from CFPQ Data (Figs. 4a-7a) have right-hand sides of three
// or more symbols, which the paper normalises automatically for the matrix
// algorithm.  All of it is removed here, on the host, before anything
// reaches the device:
//   * a right-hand side y1 y2 ... yk (k >= 3) becomes y1 H, where the helper
//     matrix H stands for the suffix y2 ... yk (H -> y2 H' and so on, down to
//     a pair); rules that share a suffix share its helper, so L(H) is the
//     concatenation of the suffix's languages whatever rule uses it;
//   * a terminal t in a binary position is replaced by a wrapper matrix T_t
//     with the single production T_t -> t (its matrix is the adjacency of
//     label t and never changes after seeding);
//   * unit rules are eliminated: for every non-terminal x and every y that x
//     reaches through unit rules (x included), x receives y's eps, terminal
//     and binary productions.  L(x) is unchanged.
#include <algorithm>
#include <cstring>
#include <functional>
#include <set>
#include <sstream>
#include <tuple>

#include "internal.h"

namespace cflr {

namespace {

struct RawRule {
    std::string lhs;
    std::vector<std::string> rhs;  // empty = eps
    int line;
};

bool valid_symbol(const std::string &s) {
    if (s.empty()) return false;
    for (char ch : s)
        if (ch == '|' || ch == '#' || (unsigned char)ch <= ' ') return false;
    return s.find("->") == std::string::npos;
}

std::vector<std::string> split_ws(const std::string &s) {
    std::vector<std::string> out;
    std::istringstream in(s);
    std::string tok;
    while (in >> tok) out.push_back(tok);
    return out;
}

}  // namespace

Lowered parse_and_lower(const char *text, size_t len) {
    std::string src(text, len);
    std::vector<RawRule> raw;
    std::vector<std::string> nts;
    std::map<std::string, uint32_t> nt_index;
    {
        std::istringstream in(src);
        std::string line;
        int lineno = 0;
        while (std::getline(in, line)) {
            ++lineno;
            auto hash = line.find('#');
            if (hash != std::string::npos) line.resize(hash);
            if (split_ws(line).empty()) continue;
            auto arrow = line.find("->");
            auto where = " (line " + std::to_string(lineno) + ")";
            if (arrow == std::string::npos) throw Error(CFLR_EPARSE, "missing '->'" + where);
            auto lhs = split_ws(line.substr(0, arrow));
            if (lhs.size() != 1 || !valid_symbol(lhs[0]) || lhs[0] == "eps")
                throw Error(CFLR_EPARSE, "left side must be one symbol" + where);
            if (!nt_index.count(lhs[0])) {
                nt_index[lhs[0]] = (uint32_t)nts.size();
                nts.push_back(lhs[0]);
            }
            std::string body = line.substr(arrow + 2);
            size_t start = 0;
            while (true) {
                size_t bar = body.find('|', start);
                auto alt = split_ws(body.substr(start, bar == std::string::npos ? std::string::npos : bar - start));
                if (alt.empty()) throw Error(CFLR_EPARSE, "empty alternative (write eps)" + where);
                for (auto &s : alt)
                    if (!valid_symbol(s)) throw Error(CFLR_EPARSE, "bad symbol '" + s + "'" + where);
                if (alt.size() == 1 && alt[0] == "eps") alt.clear();
                else if (std::find(alt.begin(), alt.end(), "eps") != alt.end())
                    throw Error(CFLR_EPARSE, "eps inside a longer right side" + where);
                raw.push_back({lhs[0], alt, lineno});
                if (bar == std::string::npos) break;
                start = bar + 1;
            }
        }
    }
    if (nts.empty()) throw Error(CFLR_EPARSE, "grammar has no productions");

    Lowered L;
    L.user_names = nts;
    L.mat_names = nts;
    std::map<std::string, uint32_t> term_index;
    auto terminal = [&](const std::string &t) {
        auto it = term_index.find(t);
        if (it != term_index.end()) return it->second;
        uint32_t id = (uint32_t)L.terminals.size();
        L.terminals.push_back(t);
        term_index[t] = id;
        return id;
    };
    auto is_nt = [&](const std::string &s) { return nt_index.count(s) > 0; };

    // wrappers for terminals in binary positions
    std::map<std::string, uint32_t> wrapper;
    auto operand = [&](const std::string &s) -> uint32_t {
        if (is_nt(s)) return nt_index[s];
        auto it = wrapper.find(s);
        if (it != wrapper.end()) return it->second;
        uint32_t m = (uint32_t)L.mat_names.size();
        L.mat_names.push_back("<" + s + ">");
        wrapper[s] = m;
        return m;
    };

    // helpers for suffixes of long right-hand sides: helper(s) has the
    // production helper(s) -> op(s[0]) op(s[1..]) (a helper for the rest
    // when it is longer than one symbol)
    std::map<std::vector<std::string>, uint32_t> helper;
    std::set<std::tuple<uint32_t, uint32_t, uint32_t>> helper_bins;
    std::function<uint32_t(const std::vector<std::string> &)> suffix_matrix =
        [&](const std::vector<std::string> &s) -> uint32_t {
        auto it = helper.find(s);
        if (it != helper.end()) return it->second;
        const uint32_t a = operand(s[0]);
        const std::vector<std::string> rest(s.begin() + 1, s.end());
        const uint32_t b = rest.size() == 1 ? operand(rest[0]) : suffix_matrix(rest);
        std::string name = "<";
        for (size_t q = 0; q < s.size(); q++) name += (q ? " " : "") + s[q];
        const uint32_t m = (uint32_t)L.mat_names.size();
        L.mat_names.push_back(name + ">");
        helper[s] = m;
        helper_bins.insert({m, a, b});
        return m;
    };

    const uint32_t U = (uint32_t)nts.size();
    // per user non-terminal: its own non-unit productions
    std::vector<std::set<std::pair<uint32_t, uint32_t>>> own_bin(U);
    std::vector<std::set<uint32_t>> own_term(U);
    std::vector<uint8_t> own_eps(U, 0);
    std::vector<std::set<uint32_t>> unit(U);  // x -> y, y non-terminal
    for (auto &r : raw) {
        uint32_t x = nt_index[r.lhs];
        if (r.rhs.empty()) {
            own_eps[x] = 1;
        } else if (r.rhs.size() == 1) {
            if (is_nt(r.rhs[0])) unit[x].insert(nt_index[r.rhs[0]]);
            else own_term[x].insert(terminal(r.rhs[0]));
        } else if (r.rhs.size() == 2) {
            uint32_t a = operand(r.rhs[0]);
            uint32_t b = operand(r.rhs[1]);
            own_bin[x].insert({a, b});
        } else {
            uint32_t a = operand(r.rhs[0]);
            uint32_t b = suffix_matrix(std::vector<std::string>(r.rhs.begin() + 1, r.rhs.end()));
            own_bin[x].insert({a, b});
        }
    }
    for (auto &w : wrapper) terminal(w.first);

    // unit closure: reach[x] = non-terminals x derives through unit rules alone
    std::set<std::tuple<uint32_t, uint32_t, uint32_t>> bins;
    std::set<std::pair<uint32_t, uint32_t>> terms;
    std::set<uint32_t> epss;
    for (uint32_t x = 0; x < U; x++) {
        std::vector<uint8_t> seen(U, 0);
        std::vector<uint32_t> stack{x};
        seen[x] = 1;
        while (!stack.empty()) {
            uint32_t y = stack.back();
            stack.pop_back();
            for (auto &ab : own_bin[y]) bins.insert({x, ab.first, ab.second});
            for (auto t : own_term[y]) terms.insert({t, x});
            if (own_eps[y]) epss.insert(x);
            for (auto z : unit[y])
                if (!seen[z]) { seen[z] = 1; stack.push_back(z); }
        }
    }
    for (auto &w : wrapper) terms.insert({term_index[w.first], w.second});
    for (auto &h : helper_bins) bins.insert(h);

    for (auto &b : bins) L.binary.push_back({std::get<0>(b), std::get<1>(b), std::get<2>(b)});
    for (auto &t : terms) L.term.push_back(t);
    L.eps.assign(epss.begin(), epss.end());
    L.wrappers = (uint32_t)wrapper.size();
    L.helpers = (uint32_t)helper.size();
    const uint32_t M = L.nmat();
    L.dynamic.assign(M, 0);
    L.slot_a.assign(M, 0);
    L.slot_b.assign(M, 0);
    for (auto &b : L.binary) {
        L.dynamic[b.c] = 1;
        L.slot_a[b.a] = 1;
        L.slot_b[b.b] = 1;
    }
    return L;
}

}  // namespace cflr
